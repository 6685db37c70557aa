"""Pins of the reference's artificial diffusion (Section 3.5): the symmetric
interior penalty form with the element-wise viscosity carried to a continuous
Q1 field (Lobatto basis).

- A_h(U, V) = -sum w J V . S(U), with S the diffusive tendency, is symmetric
  in U and V and non-negative for a fixed viscosity (its definition).
- S conserves the integral of every variable, with periodic faces and with
  slip walls (which carry no diffusive terms).
- A constant perturbation is left alone.
- Under a uniform velocity u0 the viscosity is gamma 0.5 h |u0| everywhere,
  and a sine mode decays at alpha (2 pi / L)^2: the tendency converges to
  -alpha (2 pi / L)^2 sin at order >= k - 1 (pointwise, for a second-order
  operator on an interpolant).
- Rain at rest still diffuses with its fall speed; nothing else does.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_13847_amd import synth
from exact import conservative, node_weights, periodic_mesh


def _state(mesh, seed, u=(3.0, -2.0)):
    rng = np.random.default_rng(seed)
    X = synth.node_coords(mesh)
    L = np.asarray(mesh.hi) - np.asarray(mesh.lo)
    s = [2 * np.pi * X[a] / L[a] for a in range(mesh.dim)]
    T = 285.0 + 2.0 * np.sin(s[0] + rng.uniform(0, 6)) * np.cos(s[1])
    rd = 1.1 * (1.0 + 0.01 * np.cos(s[0] - s[1]))
    rv = 0.6 * O.rho_vs(O.default_params(), 285.0) * (1.0 + 0.1 * np.sin(s[1]))
    z = np.zeros_like(T)
    uu = [u[a] * (1.0 + 0.3 * np.sin(s[(a + 1) % mesh.dim] + a)) for a in range(mesh.dim)]
    return conservative(mesh, rd, rv, z, z, T, uu)


def _oracle(mesh, bg, nvars, **over):
    P = O.default_params(g=0.0, sip_gamma=0.3, sip_sigma=10.0, **over)
    return O.Oracle(mesh, P, nvars, bg)


def _form(o, mesh, U, V, W):
    S = o.sip(U, W)
    return -np.sum(node_weights(mesh)[None] * V * S)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_form_is_symmetric_and_nonnegative(k):
    mesh = periodic_mesh((5, 4), k, L=2000.0)
    W, bg = _state(mesh, 1)
    o = _oracle(mesh, bg, 5)
    rng = np.random.default_rng(k)
    U = rng.standard_normal(W.shape)
    V = rng.standard_normal(W.shape)
    a_uv, a_vu = _form(o, mesh, U, V, W), _form(o, mesh, V, U, W)
    assert a_uv == pytest.approx(a_vu, rel=1e-11)
    assert _form(o, mesh, U, U, W) > 0.0
    assert _form(o, mesh, V, V, W) > 0.0


@pytest.mark.parametrize("walls", [False, True])
def test_every_integral_is_conserved(walls):
    if walls:
        c = synth.moist_bubble(n=(6, 4), order=3, seed=3)
        o = O.Oracle.for_case(c, sip_gamma=0.3)
        mesh, U = c.mesh, c.U.copy()
        U[2] += 5.0 * c.bg["rho_d"][synth.height_index(c.mesh)]
    else:
        mesh = periodic_mesh((5, 4), 2, L=2000.0)
        U, bg = _state(mesh, 2)
        o = _oracle(mesh, bg, 5)
    S = o.sip(U)
    W = node_weights(mesh)
    for v in range(U.shape[0]):
        assert abs(np.sum(W * S[v])) < 1e-12 * np.sum(W * np.abs(S[v])) + 1e-300, v


def test_constant_perturbation_is_untouched():
    mesh = periodic_mesh((4, 4), 3, L=2000.0)
    W, bg = _state(mesh, 4)
    o = _oracle(mesh, bg, 5)
    U = np.ones_like(W) * np.array([1e-3, 2e-4, 0.5, -0.2, 30.0])[:, None, None]
    assert np.abs(o.sip(U, W)).max() < 1e-13 * 30.0


@pytest.mark.parametrize("k,ns", [(2, (8, 16)), (3, (4, 8))])
def test_sine_mode_decays_at_alpha_k2(k, ns):
    L, u0, gam = 2000.0, 4.0, 0.3
    errs = []
    for n in ns:
        mesh = periodic_mesh((n, n), k, L=L)
        one = np.ones((mesh.ne, mesh.npe))
        W, bg = conservative(mesh, 1.1 * one, 0 * one, 0 * one, 0 * one, 290.0 * one, [u0 * one, 0 * one])
        o = _oracle(mesh, bg, 5)
        X = synth.node_coords(mesh)
        U = np.zeros_like(W)
        U[4] = np.sin(2 * np.pi * X[0] / L) * np.cos(2 * np.pi * X[1] / L)
        S = o.sip(U, W)
        alpha = gam * 0.5 * (L / n) * u0            # 2D: h^(1 - d/2) = 1, ||u||_{0,K} = u0 h
        want = -alpha * 2 * (2 * np.pi / L) ** 2 * U[4]
        errs.append(np.abs(S[4] - want).max() / np.abs(want).max())
        assert np.abs(S[:4]).max() == 0.0
    # the pointwise consistency of a second-order operator on an interpolant
    # is O(h^(k-1)); a wrong factor anywhere would stall the error instead
    assert errs[-1] < 0.15 and np.log2(errs[0] / errs[-1]) > k - 1.3, errs


def test_rain_at_rest_diffuses_with_its_fall_speed():
    mesh = periodic_mesh((4, 4), 2, L=2000.0)
    one = np.ones((mesh.ne, mesh.npe))
    X = synth.node_coords(mesh)
    rr = 1e-3 * (1.5 + np.sin(2 * np.pi * X[0] / 2000.0))
    Wst, bg = conservative(mesh, 1.1 * one, 0.004 * one, 0 * one, rr, 285.0 * one, [0 * one, 0 * one], rain=True)
    o = O.Oracle(mesh, O.default_params(g=0.0, rain=1, vr_const=5.0, sip_gamma=0.3), 6, bg)
    rng = np.random.default_rng(5)
    U = rng.standard_normal(Wst.shape)
    S = o.sip(U, Wst)
    assert np.abs(S[[0, 1, 3, 4, 5]]).max() == 0.0
    assert np.abs(S[2]).max() > 0.0


def test_diffusion_enters_the_rhs():
    mesh = periodic_mesh((4, 4), 2, L=2000.0)
    U, bg = _state(mesh, 6)
    on = _oracle(mesh, bg, 5)
    off = O.Oracle(mesh, O.default_params(g=0.0), 5, bg)
    np.testing.assert_allclose(on.rhs(U) - off.rhs(U), on.sip(U), rtol=1e-9, atol=1e-9 * np.abs(on.sip(U)).max())


def test_slip_walls_carry_no_diffusion():
    # a perturbation in the bottom element row reaches the row above only,
    # never the top row across the wall
    c = synth.moist_bubble(n=(4, 5), order=2, seed=3)
    o = O.Oracle.for_case(c, sip_gamma=0.3)
    W = c.U.copy()
    W[2] += 5.0 * c.bg["rho_d"][synth.height_index(c.mesh)]
    ez = np.arange(c.mesh.ne) // 4
    U = np.zeros_like(W)
    U[:, ez == 0] = np.random.default_rng(9).standard_normal(U[:, ez == 0].shape)
    S = o.sip(U, W)
    assert np.abs(S[:, ez == 4]).max() == 0.0
    assert np.abs(S[:, ez == 1]).max() > 0.0


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("walls", [False, True])
def test_single_element_jump_is_the_penalty(k, walls):
    # U' = 1 on one element: no gradient anywhere, so A_h(U, U) is the penalty
    # alone, sigma k^2 / h alpha |F| per interior face of that element; with
    # square elements and a uniform viscosity that is sigma k^2 alpha per face
    L, n, u0, gam, sig = 2000.0, 4, 4.0, 0.3, 10.0
    mesh = synth.Mesh(2, [n, n], [0, 0], [L, L], [0, 1 if walls else 0], k)
    one = np.ones((mesh.ne, mesh.npe))
    W, bg = conservative(mesh, 1.1 * one, 0 * one, 0 * one, 0 * one, 290.0 * one, [u0 * one, 0 * one])
    o = O.Oracle(mesh, O.default_params(g=0.0, sip_gamma=gam, sip_sigma=sig), 5, bg)
    alpha = gam * 0.5 * (L / n) * u0
    e = 1                                                  # bottom row: a wall below it if walls
    U = np.zeros_like(W)
    U[4, e] = 1.0
    got = _form(o, mesh, U, U, W)
    nfaces = 3 if walls else 4
    assert got == pytest.approx(nfaces * sig * k * k * alpha, rel=1e-12)


# ---------------------------------------------------------------------------
# the viscosity field itself: element values alpha_K and their continuous Q1
# carry by vertex means (hand-computed nodal values)
# ---------------------------------------------------------------------------
def _element_speeds_state(mesh, speeds, rain=False, w=0.0):
    """State at rest but for a horizontal velocity constant on each element
    (speeds[e]) and a uniform vertical velocity w."""
    one = np.ones((mesh.ne, mesh.npe))
    ux = np.asarray(speeds, float)[:, None] * one
    rr = 1e-3 * one if rain else 0 * one
    return conservative(mesh, 1.1 * one, 0.004 * one, 0 * one, rr, 285.0 * one, [ux, w * one], rain=rain)


def _alpha_fields(mesh, speeds, gam=0.3, rain=False, w=0.0, vr=5.0):
    W, bg = _element_speeds_state(mesh, speeds, rain=rain, w=w)
    P = O.default_params(g=0.0, sip_gamma=gam, rain=1 if rain else 0, vr_const=vr)
    o = O.Oracle(mesh, P, 6 if rain else 5, bg)
    return o.sip_alpha(W)


def _node_ref_coords(mesh):
    x = O.tables(mesh.order)[0]
    p1 = mesh.order + 1
    n = np.arange(mesh.npe)
    return x[n % p1], x[n // p1]


def test_viscosity_carry_on_a_periodic_2x2_mesh_is_the_mean():
    # every vertex of a 2 x 2 periodic mesh touches all four elements, so the
    # continuous field is the mean of the four element values everywhere
    L, gam = 2000.0, 0.3
    mesh = periodic_mesh((2, 2), 3, L=L)
    speeds = [1.0, 2.0, 3.0, 6.0]
    a0, a1 = _alpha_fields(mesh, speeds, gam)
    aK = gam * 0.5 * (L / 2) * np.asarray(speeds)        # 2D: ||u||_{0,K} = |u_K| h
    np.testing.assert_allclose(a0, np.full_like(a0, aK.mean()), rtol=1e-13)
    np.testing.assert_allclose(a1, a0, rtol=0)


def test_viscosity_carry_with_walls_interpolates_the_row_means():
    # periodic in x (2 columns), slip walls in z (2 rows): the vertices on the
    # floor touch the bottom row only, the middle vertices all four elements,
    # the lid vertices the top row only; in between, the Q1 interpolant is
    # linear in the reference height
    L, gam = 2000.0, 0.3
    mesh = synth.Mesh(2, [2, 2], [0, 0], [L, L], [0, 1], 3)
    speeds = [1.0, 2.0, 3.0, 6.0]                     # e = ex + 2 ez
    a0, _ = _alpha_fields(mesh, speeds, gam)
    c = gam * 0.5 * (L / 2)
    floor, mid, lid = c * 1.5, c * 3.0, c * 4.5
    _, eta = _node_ref_coords(mesh)
    s = 0.5 * (1.0 + eta)
    for e in range(4):
        lo, hi = (floor, mid) if e < 2 else (mid, lid)
        np.testing.assert_allclose(a0[e], (1.0 - s) * lo + s * hi, rtol=1e-13)
    # corner and mid-edge values spelled out for the bottom-left element
    p1 = mesh.order + 1
    assert a0[0][0] == pytest.approx(floor, rel=1e-13)                  # floor corner
    assert a0[0][p1 * mesh.order] == pytest.approx(mid, rel=1e-13)      # upper corner


def test_viscosity_carry_on_a_periodic_3x3_mesh_by_geometry():
    # vertex means found geometrically: a vertex at (X, Z) collects the elements
    # whose closure contains it, with periodic images; the nodal value is the
    # bilinear blend of the element's four corner means
    L, gam, n, k = 3000.0, 0.3, 3, 2
    mesh = periodic_mesh((n, n), k, L=L)
    speeds = np.array([1.0, 5.0, 2.0, 7.0, 3.0, 4.0, 9.0, 6.0, 8.0])
    a0, _ = _alpha_fields(mesh, speeds, gam)
    h = L / n
    aK = gam * 0.5 * h * speeds

    def vertex_mean(X, Z):
        vals = []
        for e in range(mesh.ne):
            ex, ez = e % n, e // n
            for sx in (-L, 0.0, L):
                for sz in (-L, 0.0, L):
                    x0, z0 = ex * h + sx, ez * h + sz
                    if x0 - 1e-9 <= X <= x0 + h + 1e-9 and z0 - 1e-9 <= Z <= z0 + h + 1e-9:
                        vals.append(aK[e])
        return np.mean(vals)

    xi, eta = _node_ref_coords(mesh)
    for e in range(mesh.ne):
        ex, ez = e % n, e // n
        corners = [[vertex_mean((ex + a) * h, (ez + b) * h) for a in (0, 1)] for b in (0, 1)]
        s, t = 0.5 * (1 + xi), 0.5 * (1 + eta)
        want = ((1 - s) * (1 - t) * corners[0][0] + s * (1 - t) * corners[0][1]
                + (1 - s) * t * corners[1][0] + s * t * corners[1][1])
        np.testing.assert_allclose(a0[e], want, rtol=1e-13)
    # the vertex means are not all alike here, so the blend is exercised
    assert np.ptp(a0) > 0.3 * np.ptp(aK)


def test_rain_viscosity_uses_the_velocity_relative_to_the_falling_rain():
    # u = (0, w) with w = 2 m/s upward and v_r = 5 m/s: the rain moves at
    # u - v_r e_z, |2 - 5| = 3 m/s (not |2 + 5| = 7); the rest moves at 2 m/s
    L, gam = 2000.0, 0.3
    mesh = periodic_mesh((3, 3), 2, L=L)
    a0, a1 = _alpha_fields(mesh, np.zeros(9), gam, rain=True, w=2.0, vr=5.0)
    c = gam * 0.5 * (L / 3)
    np.testing.assert_allclose(a0, np.full_like(a0, c * 2.0), rtol=1e-12)
    np.testing.assert_allclose(a1, np.full_like(a1, c * 3.0), rtol=1e-12)
    # downward air: |-2 - 5| = 7
    a0, a1 = _alpha_fields(mesh, np.zeros(9), gam, rain=True, w=-2.0, vr=5.0)
    np.testing.assert_allclose(a1, np.full_like(a1, c * 7.0), rtol=1e-12)
