"""Test-side constructions: exact solutions and hand-built states.

These build conservative states from primitive fields with the reference's
saturation density (pinned separately) and the paper's energy definition; they
are used to pin the reference, never by the library.
"""
import numpy as np

import oracle as O
from paper_2305_13847_amd import synth

P0 = O.default_params()
rho_vs_vec = np.vectorize(lambda T: O.rho_vs(P0, float(T)))


def conservative(mesh, rd, rv, rc, rr, T, u, bg=None, rain=False):
    """Perturbation state U (and the uniform background used) from primitives."""
    rm = rv + rc
    rho = rd + rm + rr
    m = [rho * ua for ua in u]
    ke = 0.5 * sum(ma * ma for ma in m) / rho
    E = (P0.cvd * rd + P0.cvv * rv + P0.cl * (rc + rr)) * (T - P0.Tref) \
        + rv * (P0.Lref - P0.Rv * P0.Tref) + ke
    if bg is None:
        nzq = mesh.nzq
        bg = dict(rho_d=np.full(nzq, float(np.mean(rd))), rho_m=np.full(nzq, float(np.mean(rm))),
                  rho_r=np.full(nzq, float(np.mean(rr)) if rain else 0.0),
                  E=np.full(nzq, float(np.mean(E))))
    iz = synth.height_index(mesh)
    fl = [rd - bg["rho_d"][iz], rm - bg["rho_m"][iz]]
    if rain:
        fl.append(rr - bg["rho_r"][iz])
    fl += m + [E - bg["E"][iz]]
    return np.ascontiguousarray(np.stack(fl)), bg


def periodic_mesh(n, order, L=1.0, dim=2, lo=None, basis="lobatto"):
    lo = [0.0] * dim if lo is None else lo
    return synth.Mesh(dim, list(n), list(lo), [lo[a] + L for a in range(dim)], [0] * dim, order, basis)


def _weights_1d(mesh):
    """Quadrature weights of the mesh's nodes: Lobatto, or Gauss for the modal basis."""
    if getattr(mesh, "basis", "lobatto") == "gauss":
        return O.gauss_tables(mesh.order)[1]
    return O.tables(mesh.order)[1]


def vortex(mesh, t, u0=(1.0, 0.5), beta=2.0, rho_inf=1.0, p_inf=1e5, r0=None):
    """Dry isentropic vortex translated by u0 t (exact solution of dry Euler).

    With rho_m = rho_r = 0 the moist system is the Euler system with
    gamma = 1 + R_d/c_vd (the energy's T_ref offset is a multiple of the
    conserved density).  Lengths scale with r0, speeds with sqrt(p/rho).
    """
    gam = 1.0 + P0.Rd / P0.cvd
    X = synth.node_coords(mesh)
    L = np.asarray(mesh.hi) - np.asarray(mesh.lo)
    ctr = np.asarray(mesh.lo) + 0.5 * L
    r0 = L[0] / 10.0 if r0 is None else r0
    cs = np.sqrt(p_inf / rho_inf)
    # periodic distance from the translated centre
    dx = []
    for a in range(2):
        s = X[a] - ctr[a] - u0[a] * cs * t
        s = (s + 0.5 * L[a]) % L[a] - 0.5 * L[a]
        dx.append(s / r0)
    r2 = dx[0] ** 2 + dx[1] ** 2
    f = np.exp(0.5 * (1.0 - r2))
    du = [-beta / (2 * np.pi) * dx[1] * f * cs, beta / (2 * np.pi) * dx[0] * f * cs]
    th = 1.0 - (gam - 1.0) * beta ** 2 / (8 * gam * np.pi ** 2) * np.exp(1.0 - r2)
    rho = rho_inf * th ** (1.0 / (gam - 1.0))
    p = p_inf * th * rho / rho_inf
    T = p / (rho * P0.Rd)
    u = [u0[0] * cs + du[0], u0[1] * cs + du[1]]
    z = np.zeros_like(rho)
    return rho, z, z, z, T, u


def moist_contact(mesh, t, u0=(20.0, 10.0), p=8e4, Tm=285.0, dT=4.0, cloud=3e-3):
    """Saturated cloudy contact translated by u0 t: uniform p and u.

    T varies smoothly, the vapour is at saturation, cloud water varies and the
    dry density closes the equation of state, so every field is advected.
    """
    return moist_contact_at(synth.node_coords(mesh), mesh.lo, np.asarray(mesh.hi) - np.asarray(mesh.lo), t, u0,
                            p, Tm, dT, cloud)


def moist_contact_at(X, lo, L, t, u0=(20.0, 10.0), p=8e4, Tm=285.0, dT=4.0, cloud=3e-3):
    """The moist contact at the points X = [x, z] of a periodic box lo + [0, L]."""
    s = [2 * np.pi * (X[a] - lo[a] - u0[a] * t) / L[a] for a in range(2)]
    T = Tm + dT * np.sin(s[0]) * np.cos(s[1])
    rc = cloud * (1.2 + np.cos(s[0] + 2 * s[1]))
    rv = rho_vs_vec(T)
    rd = (p / T - rv * P0.Rv) / P0.Rd
    z = np.zeros_like(T)
    return rd, rv, rc, z, T, [u0[0] + z, u0[1] + z]


def l2(mesh, f):
    """Discrete L2 norm with the nodes' quadrature weights and the element Jacobian."""
    w = _weights_1d(mesh)
    p1 = mesh.order + 1
    W = np.ones(p1 ** mesh.dim)
    for a in range(mesh.dim):
        idx = (np.arange(p1 ** mesh.dim) // (p1 ** a)) % p1
        W *= w[idx]
    J = np.prod(mesh.h) / 2 ** mesh.dim
    return np.sqrt(np.sum(W[None, :] * J * f * f))


def node_weights(mesh):
    w = _weights_1d(mesh)
    p1 = mesh.order + 1
    W = np.ones(p1 ** mesh.dim)
    for a in range(mesh.dim):
        idx = (np.arange(p1 ** mesh.dim) // (p1 ** a)) % p1
        W *= w[idx]
    return W[None, :] * np.prod(mesh.h) / 2 ** mesh.dim * np.ones((mesh.ne, 1))


def tri_conservative(rd, rv, rc, rr, T, u, rain=False):
    """Conservative fields (rho_d, rho_m, [rho_r], m_x, m_z, E) from primitives."""
    rm = rv + rc
    rho = rd + rm + rr
    m = [rho * ua for ua in u]
    ke = 0.5 * sum(ma * ma for ma in m) / rho
    E = (P0.cvd * rd + P0.cvv * rv + P0.cl * (rc + rr)) * (T - P0.Tref) \
        + rv * (P0.Lref - P0.Rv * P0.Tref) + ke
    return [rd, rm] + ([rr] if rain else []) + m + [E]


def tri_l2(o, C):
    """L2 norm of fields C (nf, ne, np) on the triangulation of o: the basis is
    orthonormal on the unit triangle, so |f|^2 = sum_e det A_e sum_m c_m^2."""
    xy = o.mesh.xy
    det = (xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1]) \
        - (xy[:, 2, 0] - xy[:, 0, 0]) * (xy[:, 1, 1] - xy[:, 0, 1])
    return np.sqrt(np.sum(det[None, :, None] * C * C, axis=(1, 2)))
