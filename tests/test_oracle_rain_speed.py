"""Pins of the reference's terminal rain speed in the COSMO mode (Section 2.1)
and of the sedimentation it drives.

The paper takes the mean terminal velocity of rain from the COSMO warm-rain
scheme: rain drops of diameter D follow the exponential (Marshall-Palmer)
size distribution N(D) = N_0 exp(-lambda D), fall at v(D) = v_0 D^(1/2) and
weigh (pi/6) rho_w D^3; v_r is the mass-weighted mean fall speed, and
lambda is fixed by the rain density rho_r.  The pins evaluate that
definition by numerical quadrature (the closed form is not used), with
N_0 = 8e6 m^-4, v_0 = 130 m^(1/2)/s and rho_w = 1000 kg/m^3:

- v_r at rho_r = 1e-3 and 1e-4 kg/m^3 (5.326 and 3.994 m/s);
- the scaling v_r(2^8 rho_r) = 2 v_r(rho_r), which fixes the exponent 1/8;
- with rain at rest, sedimentation lowers the rain-mass centroid at the
  mass-weighted v_r, and rain mass leaves through the floor at rho_r v_r(rho_r)
  (semi-discrete identities of the perturbation system, Section 2.3).
"""
import numpy as np
import pytest
from scipy import integrate, optimize

import oracle as O
from paper_2305_13847_amd import synth
from exact import conservative, node_weights, rho_vs_vec

N0, V0, RHO_W = 8.0e6, 130.0, 1000.0


def _mass(lam):
    # integral of (pi/6) rho_w D^3 N0 exp(-lam D) over the drop sizes
    f = lambda D: (np.pi / 6.0) * RHO_W * D ** 3 * N0 * np.exp(-lam * D)
    return integrate.quad(f, 0.0, 80.0 / lam, epsabs=0.0, epsrel=1e-13, limit=200)[0]


def v_mean_quadrature(rho_r):
    """Mass-weighted mean fall speed of the exponential size distribution whose
    mass content is rho_r, by numerical quadrature and root finding."""
    lam = optimize.brentq(lambda l: np.log(_mass(l) / rho_r), 10.0, 1e6, xtol=1e-14, rtol=1e-15)
    f = lambda D: V0 * np.sqrt(D) * (np.pi / 6.0) * RHO_W * D ** 3 * N0 * np.exp(-lam * D)
    flux = integrate.quad(f, 0.0, 80.0 / lam, epsabs=0.0, epsrel=1e-13, limit=200)[0]
    return flux / _mass(lam)


def _oracle_vr(rho_r):
    """v_r of the reference at rain density rho_r: F_z[rho_r'] = -rho_r v_r at rest."""
    mesh = synth.Mesh(2, [1, 1], [0, 0], [1e3, 1e3], [0, 0], 1)
    bg = dict(rho_d=np.full(mesh.nzq, 1.1), rho_m=np.full(mesh.nzq, 0.01), rho_r=np.zeros(mesh.nzq),
              E=np.full(mesh.nzq, 2.3e5))
    o = O.Oracle(mesh, O.default_params(rain=1, vr_mode=1, g=0.0), 6, bg)
    Uq = np.zeros(6)
    Uq[2] = rho_r
    F, _, _ = o.point(Uq, 0)
    return -F[1, 2] / rho_r


def test_worked_values():
    for rr, want in ((1e-3, 5.326), (1e-4, 3.994)):
        vq = v_mean_quadrature(rr)
        assert vq == pytest.approx(want, abs=5e-4)
        assert _oracle_vr(rr) == pytest.approx(vq, rel=1e-9)


@pytest.mark.parametrize("rr", [3e-6, 2e-5, 7e-4, 4e-3])
def test_matches_the_size_distribution_mean(rr):
    assert _oracle_vr(rr) == pytest.approx(v_mean_quadrature(rr), rel=1e-9)


def test_exponent_one_eighth():
    for rr in (1e-6, 1e-4):
        assert _oracle_vr(rr * 2.0 ** 8) == pytest.approx(2.0 * _oracle_vr(rr), rel=1e-12)
        assert v_mean_quadrature(rr * 2.0 ** 8) == pytest.approx(2.0 * v_mean_quadrature(rr), rel=1e-9)


def test_no_rain_no_speed():
    assert _oracle_vr(1e-300) < 1e-30
    mesh = synth.Mesh(2, [1, 1], [0, 0], [1e3, 1e3], [0, 0], 1)
    bg = dict(rho_d=np.full(mesh.nzq, 1.1), rho_m=np.full(mesh.nzq, 0.01), rho_r=np.zeros(mesh.nzq),
              E=np.full(mesh.nzq, 2.3e5))
    o = O.Oracle(mesh, O.default_params(rain=1, vr_mode=1, g=0.0), 6, bg)
    Uq = np.zeros(6)
    Uq[2] = -1e-4                                   # negative rain: clamped, no fall speed
    _, _, lam = o.point(Uq, 0)
    assert lam[1] == lam[0]                         # at rest: lambda_z - lambda_x = |v_r|
    Uq[2] = 1e-3
    _, _, lam = o.point(Uq, 0)
    assert lam[1] - lam[0] == pytest.approx(v_mean_quadrature(1e-3), rel=1e-9)


def _rain_at_rest(mesh, touching_floor):
    X = synth.node_coords(mesh)
    T = 290.0 - 6.5e-3 * X[-1]
    rd = 1.1 * np.exp(-X[-1] / 8e3)
    rvs = rho_vs_vec(T)
    rm = rvs * (1.0 + 0.2 * np.sin(X[0] / 700.0))
    rv = np.minimum(rm, rvs)
    zc = 0.0 if touching_floor else 2.5e3
    r = np.sqrt(((X[0] - 3e3) / 1.5e3) ** 2 + ((X[-1] - zc) / 1e3) ** 2)
    rr = 2e-3 * np.cos(0.5 * np.pi * np.minimum(r, 1.0)) ** 2 + 1e-5
    z0 = np.zeros_like(T)
    bg = dict(rho_d=np.zeros(mesh.nzq), rho_m=np.zeros(mesh.nzq), rho_r=np.zeros(mesh.nzq),
              E=np.zeros(mesh.nzq))
    U, _ = conservative(mesh, rd, rv, rm - rv, rr, T, [z0, z0], bg=bg, rain=True)
    iz = synth.height_index(mesh)
    for key, v in (("rho_d", 0), ("rho_m", 1), ("rho_r", 2), ("E", 5)):
        for q in range(mesh.nzq):
            bg[key][q] = U[v][iz == q].mean()
        U[v] -= bg[key][iz]
    return U, bg, rr


def _vr_field(rr):
    # v_r = C rho_r^(1/8) with C from the quadrature at one density (the
    # exponent is pinned separately)
    C = v_mean_quadrature(1e-3) / 1e-3 ** 0.125
    return C * np.maximum(rr, 0.0) ** 0.125


def test_sedimentation_moves_the_centroid_at_the_mass_weighted_speed():
    # at rest and away from the walls: d/dt sum wJ z (rho_m' + rho_r')
    #   = -sum wJ rho_r v_r(rho_r)
    mesh = synth.Mesh(2, [6, 6], [0, 0], [6e3, 6e3], [0, 1], 2)
    U, bg, rr = _rain_at_rest(mesh, touching_floor=False)
    o = O.Oracle(mesh, O.default_params(rain=1, vr_mode=1, g=0.0), 6, bg)
    R = o.rhs(U)
    W = node_weights(mesh)
    z = synth.node_heights(mesh)[synth.height_index(mesh)]
    lhs = np.sum(W * z * (R[1] + R[2]))
    # the tiny rain floor (1e-5) reaches the walls: take the floor and lid
    # fluxes out of the identity with the outflow below
    x, w, _, _ = O.tables(mesh.order)
    p1 = mesh.order + 1
    wf = (w[np.arange(mesh.npe) % p1] * 0.5 * mesh.h[0])[None, :] * np.ones((mesh.ne, 1))
    top = (np.arange(mesh.ne) >= mesh.ne - mesh.n[0])[:, None] & (np.arange(mesh.npe) // p1 == mesh.order)[None, :]
    lid = np.sum((wf * z * rr * _vr_field(rr))[top])   # rain entering through the lid at z = H
    assert lhs == pytest.approx(-np.sum(W * rr * _vr_field(rr)) + lid, rel=1e-9)


def test_rain_leaves_through_the_floor_at_rho_r_v_r():
    mesh = synth.Mesh(2, [6, 4], [0, 0], [6e3, 4e3], [0, 1], 3)
    U, bg, rr = _rain_at_rest(mesh, touching_floor=True)
    o = O.Oracle(mesh, O.default_params(rain=1, vr_mode=1, g=9.81), 6, bg)
    R = o.rhs(U)
    W = node_weights(mesh)
    x, w, _, _ = O.tables(mesh.order)
    p1 = mesh.order + 1
    floor = (np.arange(mesh.ne) < mesh.n[0])[:, None] & (np.arange(mesh.npe) // p1 == 0)[None, :]
    top = (np.arange(mesh.ne) >= mesh.ne - mesh.n[0])[:, None] & (np.arange(mesh.npe) // p1 == mesh.order)[None, :]
    wf = (w[np.arange(mesh.npe) % p1] * 0.5 * mesh.h[0])[None, :] * np.ones((mesh.ne, 1))
    flux = wf * rr * _vr_field(rr)
    out = np.sum(flux[floor]) - np.sum(flux[top])
    assert np.sum(W * (R[1] + R[2])) == pytest.approx(-out, rel=1e-9)
    # and the reference's own wall-flux diagnostic agrees
    assert o.mass(U)[2] == pytest.approx(out, rel=1e-9)
