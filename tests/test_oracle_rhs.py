"""Pins of the reference right-hand side by invariants the paper's system fixes.

Each check would fail on a plausible slip in the reference (a dropped term, a
wrong sign, a wrong axis or index): constant states, rest states, rotation and
mirror symmetry, 2D = y-independent 3D, semi-discrete energy and rain-mass
identities, conservation over RK steps, hydrostatic balance and the Kessler
sources' structure.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_13847_amd import synth
from exact import (P0, conservative, node_weights, periodic_mesh, rho_vs_vec)


def make(mesh, nvars, bg, **over):
    P = O.default_params(**over)
    return O.Oracle(mesh, P, nvars, bg)


def test_dry_sound_speed_and_pure_vapour_limit():
    mesh = periodic_mesh((2, 2), 2)
    for (rd, rv) in ((1.2, 0.0), (0.0, 0.01)):
        n = mesh.ne * mesh.npe
        T = np.full((mesh.ne, mesh.npe), 290.0)
        U, bg = conservative(mesh, rd + 0 * T, rv + 0 * T, 0 * T, 0 * T, T, [0 * T, 0 * T])
        o = make(mesh, 5, bg, g=0.0)
        s = o.split_field(U)
        if rd > 0:
            gam, p, rho = 1 + P0.Rd / P0.cvd, rd * P0.Rd * 290.0, rd
        else:
            gam, p, rho = 1 + P0.Rv / P0.cvv, rv * P0.Rv * 290.0, rv
        assert np.allclose(s["c_m"], np.sqrt(gam * p / rho), rtol=1e-13)
        assert abs(1 + P0.Rd / P0.cvd - 1.39979) < 1e-5


def test_constant_state_is_steady():
    mesh = periodic_mesh((4, 3), 3, L=1000.0)
    T = np.full((mesh.ne, mesh.npe), 288.0)
    rvs = rho_vs_vec(288.0)
    U, bg = conservative(mesh, 1.1 + 0 * T, rvs + 0 * T, 2e-3 + 0 * T, 0 * T, T,
                         [12.0 + 0 * T, -7.0 + 0 * T])
    o = make(mesh, 5, bg, g=0.0)
    R = o.rhs(U)
    scale = [1.1 * 12 / 1000, 0.02 * 12 / 1000, 1e5 / 1000, 1e5 / 1000, 3e5 * 12 / 1000]
    for v in range(5):
        assert np.max(np.abs(R[v])) < 1e-12 * scale[v] * 1e3


@pytest.mark.parametrize("rain", [0, 1])
def test_rest_state_rhs_is_exactly_zero(rain):
    if rain:
        c = synth.warm_rain_3d(n=(3, 2, 4), noise=0)
    else:
        c = synth.moist_bubble(n=(6, 5), order=3, noise=0)
    o = O.Oracle.for_case(c)
    R = o.rhs(np.zeros_like(c.U))
    if rain:
        # the cloudy background autoconverts: only the water sources survive
        assert np.all(R[[0, 3, 4, 5, 6]] == 0.0)
        assert np.all(R[1] + R[2] == 0.0) and np.any(R[2] > 0)
    else:
        assert np.all(R == 0.0)


def _random_periodic_state(mesh, seed, rain=False):
    rng = np.random.default_rng(seed)
    X = synth.node_coords(mesh)
    L = [mesh.hi[a] - mesh.lo[a] for a in range(mesh.dim)]

    def field():
        s = 0 * X[0]
        for _ in range(3):
            kv = rng.integers(1, 3, size=mesh.dim)
            s += rng.uniform(0.5, 1) * np.sin(sum(2 * np.pi * kv[a] * X[a] / L[a] for a in range(mesh.dim))
                                              + rng.uniform(0, 6.28))
        return s / np.max(np.abs(s))

    T = 285.0 + 3 * field()
    rd = 1.1 * (1 + 0.01 * field())
    rvs = rho_vs_vec(T)
    rm = rvs * (1.0 + 0.3 * field())
    rv = np.minimum(rm, rvs)
    rr = 1e-3 * (1.2 + field()) if rain else 0 * T
    u = [5.0 * field() for _ in range(mesh.dim)]
    return conservative(mesh, rd, rv, rm - rv, rr, T, u, rain=rain)


def test_rotation_covariance_2d():
    # g = 0 and periodic in both axes: swapping x and z must swap the momentum
    # components and transpose the element and node grids
    k, n = 3, 4
    mesh = periodic_mesh((n, n), k, L=2000.0)
    U, bg = _random_periodic_state(mesh, 3)
    o = make(mesh, 5, bg, g=0.0)
    R = o.rhs(U)
    p1 = k + 1

    def transpose(A):
        B = A.reshape(A.shape[0], n, n, p1, p1)          # v, ez, ex, j, i
        return B.transpose(0, 2, 1, 4, 3).reshape(A.shape)
    Ut = transpose(U)[[0, 1, 3, 2, 4]]
    Rt = o.rhs(Ut)
    assert np.allclose(Rt, transpose(R)[[0, 1, 3, 2, 4]], rtol=1e-11, atol=1e-11 * np.abs(R).max())


def test_mirror_symmetry_with_walls_and_gravity():
    c = synth.moist_bubble(n=(8, 4), order=3, noise=0, centre=(10e3, 2e3))
    o = O.Oracle.for_case(c)
    k, (nx, nz) = 3, c.mesh.n
    p1 = k + 1

    def mirror(A):
        B = A.reshape(A.shape[:-2] + (nz, nx, p1, p1))[..., ::-1, :, ::-1]
        return B.reshape(A.shape)
    U = c.U.copy()
    U[2] = 0.3 * U[4] / np.abs(U[4]).max()              # some antisymmetric x-momentum
    U[2] = U[2] - mirror(U[2])
    U[3] = 0.2 * (U[4] + mirror(U[4])) / np.abs(U[4]).max()
    R = o.rhs(U)
    sgn = np.array([1, 1, -1, 1, 1])[:, None, None]
    Rm = sgn * mirror(R)
    assert np.allclose(R, Rm, rtol=1e-11, atol=1e-11 * np.abs(R).max(axis=(1, 2), keepdims=True))


def test_3d_reduces_to_2d():
    k = 2
    m2 = periodic_mesh((4, 4), k, L=1500.0)
    U2, bg = _random_periodic_state(m2, 5)
    m3 = synth.Mesh(3, [4, 3, 4], [0, 0, 0], [1500.0, 900.0, 1500.0], [0, 0, 0], k)
    p1 = k + 1
    # 3D state constant in y: e3 = ex + 4 (ey + 3 ez); n3 = i + p1 (j + p1 l)
    U3 = np.zeros((6, m3.ne, m3.npe))
    A = U2.reshape(5, 4, 4, p1, p1)                     # v, ez, ex, l, i
    for ey in range(3):
        for j in range(p1):
            for vv, v3 in zip(range(5), [0, 1, 2, 4, 5]):
                B = U3[v3].reshape(4, 3, 4, p1, p1, p1)  # ez, ey, ex, l, j, i
                B[:, ey, :, :, j, :] = A[vv]
    o2 = make(m2, 5, bg, g=0.0)
    o3 = make(m3, 6, bg, g=0.0)
    R2 = o2.rhs(U2).reshape(5, 4, 4, p1, p1)
    R3 = o3.rhs(U3).reshape(6, 4, 3, 4, p1, p1, p1)
    for vv, v3 in zip(range(5), [0, 1, 2, 4, 5]):
        for ey in range(3):
            for j in range(p1):
                assert np.allclose(R3[v3][:, ey, :, :, j, :], R2[vv], rtol=1e-12,
                                   atol=1e-12 * np.abs(R2[vv]).max())
    assert np.max(np.abs(R3[3])) < 1e-9 * np.abs(R2[3]).max()


def _heights(mesh):
    return synth.node_heights(mesh)[synth.height_index(mesh)]


def test_energy_with_potential_is_invariant_without_rain():
    # (E' + g z rho') is conserved by the semi-discrete system with slip walls
    c = synth.moist_bubble(n=(6, 5), order=3)
    c.U[2] += 0.5 * c.bg["rho_d"][synth.height_index(c.mesh)] * np.sin(
        synth.node_coords(c.mesh)[1] / 1e3)
    o = O.Oracle.for_case(c)
    R = o.rhs(c.U)
    W = node_weights(c.mesh)
    z = _heights(c.mesh)
    lhs = np.sum(W * (R[4] + c.g * z * (R[0] + R[1])))
    scale = np.sum(W * np.abs(R[4]))
    assert abs(lhs) < 1e-12 * scale


def _rain_state(mesh, touching_floor, seed=8):
    rng = np.random.default_rng(seed)
    X = synth.node_coords(mesh)
    T = 290.0 - 6.5e-3 * X[-1]
    rd = 1.1 * np.exp(-X[-1] / 8e3)
    rvs = rho_vs_vec(T)
    rm = rvs * (1.0 + 0.2 * np.sin(X[0] / 700.0))
    rv = np.minimum(rm, rvs)
    zc = 0.0 if touching_floor else 2.5e3
    r = np.sqrt(((X[0] - 3e3) / 1.5e3) ** 2 + ((X[-1] - zc) / 1e3) ** 2)
    rr = 2e-3 * np.cos(0.5 * np.pi * np.minimum(r, 1.0)) ** 2
    u = [3.0 + 2 * np.cos(X[-1] / 500.0), (0.0 if not touching_floor else 0.5) * np.sin(X[0] / 800.0) * 0]
    bg = dict(rho_d=np.zeros(mesh.nzq), rho_m=np.zeros(mesh.nzq), rho_r=np.zeros(mesh.nzq),
              E=np.zeros(mesh.nzq))
    # background: the column average of the state (any background works)
    U, _ = conservative(mesh, rd, rv, rm - rv, rr, T, u, bg=bg, rain=True)
    iz = synth.height_index(mesh)
    for key, v in (("rho_d", 0), ("rho_m", 1), ("rho_r", 2), ("E", 5)):
        for q in range(mesh.nzq):
            bg[key][q] = U[v][iz == q].mean()
        U[v] -= bg[key][iz]
    return U, bg, T


def test_rain_falls_at_terminal_speed():
    # at rest, sum wJ z (R_r + R_m) = -v_r sum wJ rho_r: sedimentation moves the
    # rain-mass centroid down at v_r (sources sum to zero)
    mesh = synth.Mesh(2, [6, 6], [0, 0], [6e3, 6e3], [0, 1], 2)
    U, bg, _ = _rain_state(mesh, touching_floor=False)
    U[3] = 0.0
    U[4] = 0.0
    P = O.default_params(rain=1, vr_const=5.0)
    o = O.Oracle(mesh, P, 6, bg)
    R = o.rhs(U)
    W = node_weights(mesh)
    z = _heights(mesh)
    rr = U[2] + bg["rho_r"][synth.height_index(mesh)]
    lhs = np.sum(W * z * (R[1] + R[2]))
    assert lhs == pytest.approx(-5.0 * np.sum(W * rr), rel=1e-10)


def test_rain_mass_momentum_energy_leave_through_the_floor():
    # semi-discrete identities with rain touching the bottom wall:
    #   d/dt sum wJ (rho_m'+rho_r')        = -sum_floor wf rho_r v_r
    #   d/dt sum wJ m_x                    = -sum_floor wf rho_r v_r u_x
    #   d/dt sum wJ (E' + g z rho')        = -g v_r sum wJ rho_r
    #                                        -sum_floor wf (c_l (T-T_ref) + u.u/2) rho_r v_r
    mesh = synth.Mesh(2, [6, 4], [0, 0], [6e3, 4e3], [0, 1], 3)
    U, bg, _ = _rain_state(mesh, touching_floor=True)
    U[4] = 0.0                                          # no vertical momentum
    vr, g = 5.0, 9.81
    P = O.default_params(rain=1, vr_const=vr, g=g)
    o = O.Oracle(mesh, P, 6, bg)
    R = o.rhs(U)
    W = node_weights(mesh)
    iz = synth.height_index(mesh)
    z = _heights(mesh)
    s = o.split_field(U)
    rr = U[2] + bg["rho_r"][iz]
    rho = U[0] + U[1] + U[2] + (bg["rho_d"] + bg["rho_m"] + bg["rho_r"])[iz]
    ux = U[3] / rho
    x, w, _, _ = O.tables(mesh.order)
    p1 = mesh.order + 1
    floor = (np.arange(mesh.ne) < mesh.n[0])[:, None] & (np.arange(mesh.npe) // p1 == 0)[None, :]
    wf = (w[np.arange(mesh.npe) % p1] * 0.5 * mesh.h[0])[None, :] * np.ones((mesh.ne, 1))
    out_w = np.sum((wf * rr * vr)[floor])
    assert np.sum(W * (R[1] + R[2])) == pytest.approx(-out_w, rel=1e-10)
    assert np.sum(W * R[3]) == pytest.approx(-np.sum((wf * rr * vr * ux)[floor]), rel=1e-9)
    X = P0.cl * (s["T"] - P0.Tref) + 0.5 * ux * ux
    rhs_E = -g * vr * np.sum(W * rr) - np.sum((wf * X * rr * vr)[floor])
    lhs_E = np.sum(W * (R[5] + g * z * (R[0] + R[1] + R[2])))
    assert lhs_E == pytest.approx(rhs_E, rel=1e-9)


def test_conservation_over_rk_steps():
    c = synth.warm_rain_3d(n=(3, 3, 3), nsteps=3)
    o = O.Oracle.for_case(c)
    m0 = o.mass(c.U)
    U1, outflow = o.rk(c.U, c.dt * 2, 3)
    m1 = o.mass(U1)
    W = node_weights(c.mesh)
    scale_d = np.sum(W * (c.bg["rho_d"][synth.height_index(c.mesh)]))
    assert abs(m1[0] - m0[0]) < 1e-14 * scale_d
    assert (m1[1] - m0[1]) == pytest.approx(-outflow, rel=1e-9)
    assert outflow != 0.0


def test_kessler_sources_structure():
    # spatially uniform state, g = 0, periodic: dU/dt = G at every node
    mesh = periodic_mesh((1, 1), 1)
    P = O.default_params(rain=1, g=0.0)
    T0 = 283.0
    rvs = O.rho_vs(P, T0)
    ones = np.ones((1, 4))
    cases = {
        "saturated_with_rain": (rvs * 1.2, 1e-3),
        "saturated_no_rain": (rvs * 1.2, 0.0),
        "unsaturated_with_rain": (rvs * 0.8, 1e-3),
    }
    for name, (rm, rr) in cases.items():
        rv = min(rm, rvs)
        U, bg = conservative(mesh, 1.0 * ones, rv * ones, (rm - rv) * ones, rr * ones, T0 * ones,
                             [0 * ones, 0 * ones], rain=True)
        o = O.Oracle(mesh, P, 6, bg)
        R = o.rhs(U)
        s = o.split_field(U)
        Gm, Gr = R[1, 0, 0], R[2, 0, 0]
        assert Gm + Gr == pytest.approx(0.0, abs=1e-18)
        assert np.all(R[3:] == 0)
        rc = s["rho_c"][0, 0]
        if name == "saturated_no_rain":
            assert Gr == pytest.approx(1e-3 * rc, rel=1e-12)     # autoconversion only
        if name == "saturated_with_rain":
            # no evaporation in saturated air: autoconversion + accretion
            assert Gr == pytest.approx(1e-3 * rc + 1.72 * rc * rr ** 0.875, rel=1e-12)
        if name == "unsaturated_with_rain":
            # worked value of the evaporation rate (COSMO form, Section 2.1)
            T = s["T"][0, 0]
            dv = O.rho_vs(P, T) - rm
            Sev = (3.86e-3 - 9.41e-5 * (T - P.Tref)) * (1 + 9.1 * rr ** 0.1875) * dv * rr ** 0.5
            assert Gm == pytest.approx(Sev, rel=1e-12) and Gm > 0


@pytest.mark.parametrize("k", [2, 3])
def test_hydrostatic_perturbation_is_balanced(k):
    # background and background+perturbation are two isothermal hydrostatic dry
    # atmospheres; the momentum tendency -dp'/dz - rho' g must vanish as h -> 0
    g, H = 9.81, 10e3
    errs = []
    for nz in (4, 8, 16):
        mesh = synth.Mesh(2, [2, nz], [0, 0], [2e3, H], [0, 1], k)
        z = synth.node_heights(mesh)
        T1, T2 = 280.0, 284.0
        rho1 = 1.2 * np.exp(-g * z / (P0.Rd * T1))
        p1_ = rho1 * P0.Rd * T1
        rho2 = p1_[0] / (P0.Rd * T2) * np.exp(-g * z / (P0.Rd * T2))
        E1 = P0.cvd * rho1 * (T1 - P0.Tref)
        E2 = P0.cvd * rho2 * (T2 - P0.Tref)
        bg = dict(rho_d=rho1, rho_m=0 * z, rho_r=0 * z, E=E1)
        o = make(mesh, 5, bg, g=g)
        iz = synth.height_index(mesh)
        U = np.zeros((5, mesh.ne, mesh.npe))
        U[0] = (rho2 - rho1)[iz]
        U[4] = (E2 - E1)[iz]
        R = o.rhs(U)
        assert np.all(R[[0, 1, 2, 4]] == 0.0) or np.max(np.abs(R[[0, 1, 2, 4]])) < 1e-12
        errs.append(np.max(np.abs(R[3])) / (g * np.max(np.abs(U[0]))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < errs[0]
    assert rates[-1] > k - 0.3


def _two_rain_states(seed=21):
    mesh = synth.Mesh(2, [2, 2], [0, 0], [2e3, 2e3], [0, 1], 2)
    rng = np.random.default_rng(seed)
    P = O.default_params(rain=1, vr_const=5.0, g=9.81)
    bg = dict(rho_d=np.full(mesh.nzq, 1.1), rho_m=np.full(mesh.nzq, 0.012),
              rho_r=np.full(mesh.nzq, 5e-4), E=np.full(mesh.nzq, 2.5e4))
    o = O.Oracle(mesh, P, 6, bg)
    Us = []
    for _ in range(2):
        Uq = np.array([0.01, 0.004, 3e-4, 0, 0, 3e3]) * rng.uniform(-1, 1, 6)
        Uq[3:5] = rng.uniform(-8, 8, 2)
        Us.append(Uq)
    return o, Us


def test_face_flux_consistency_and_antisymmetry():
    o, (Ua, Ub) = _two_rain_states()
    for j in (0, 1):
        F, _, _ = o.point(Ua, 2)
        assert np.allclose(o.face(Ua, 2, Ua, 2, j), F[j], rtol=1e-14, atol=1e-12)
        if j == 1:
            continue          # falling rain breaks the up/down mirror symmetry
        # swapping the sides and the normal flips the flux; reflecting momentum
        # in e_j turns U(+n) into U(-n)
        flip = np.ones(6)
        flip[3 + j] = -1.0
        Fab = o.face(Ua, 2, Ub, 2, j)
        Fba = o.face(flip * Ub, 2, flip * Ua, 2, j)
        assert np.allclose(Fab, -flip * Fba, rtol=1e-12, atol=1e-12 * np.abs(Fab).max())


def test_face_dissipation_is_max_wave_speed():
    # F*(U-, U+) - (F(U-) + F(U+)).n/2 = Lambda/2 (U- - U+) with
    # Lambda = max over sides of |u.n| + |v_r e_z.n| + c_m
    o, (Ua, Ub) = _two_rain_states(5)
    for j in (0, 1):
        Fa, _, la = o.point(Ua, 2)
        Fb, _, lb = o.point(Ub, 2)
        diss = o.face(Ua, 2, Ub, 2, j) - 0.5 * (Fa[j] + Fb[j])
        Lam = 2 * diss / (Ua - Ub)
        assert np.allclose(Lam, Lam[0], rtol=1e-8)
        s = o.split_field(np.tile(np.stack([Ua, Ub], 1)[:, :, None], (1, 2, 9))[:, :, :])
        rho = lambda Uq: Uq[0] + Uq[1] + Uq[2] + 1.1 + 0.012 + 5e-4
        speeds = []
        for Uq, cm in ((Ua, s["c_m"][0, 0]), (Ub, s["c_m"][1, 0])):
            speeds.append(abs(Uq[3 + j] / rho(Uq)) + (5.0 if j == 1 else 0.0) + cm)
        assert Lam[0] == pytest.approx(max(speeds), rel=1e-10)


def test_moist_sound_speed_worked_example():
    # c_m^2 = gamma_m p / rho with gamma_m in the paper's mixing-ratio form,
    # liquid (cloud + rain) included in the heat capacity
    mesh = periodic_mesh((1, 1), 1)
    P = O.default_params(rain=1, g=0.0)
    T0 = 287.0
    rvs = O.rho_vs(P, T0)
    ones = np.ones((1, 4))
    rd, rc, rr = 1.05, 2.5e-3, 1.5e-3
    U, bg = conservative(mesh, rd * ones, rvs * ones, rc * ones, rr * ones, T0 * ones,
                         [0 * ones, 0 * ones], rain=True)
    o = O.Oracle(mesh, P, 6, bg)
    s = o.split_field(U)
    qv, qc, qr = rvs / rd, rc / rd, rr / rd
    cv = P0.cvd + qv * P0.cvv + (qc + qr) * P0.cl
    gam = (cv + P0.Rd + qv * P0.Rv) / cv
    p = (rd * P0.Rd + rvs * P0.Rv) * T0
    assert s["c_m"][0, 0] == pytest.approx(np.sqrt(gam * p / (rd + rvs + rc + rr)), rel=1e-12)
