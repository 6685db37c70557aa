"""Pins of the reference on triangles (Section 3.1 P^k space; the Duffy-mapped
Gauss-Legendre rule of the footnote in Section 3.4).

* The volume rule integrates every monomial r^a s^b of degree <= 2k+1 over the
  unit triangle exactly: a! b! / (a + b + 2)!.
* The basis is orthonormal under that rule, spans P^k (every monomial of degree
  <= k is reproduced by its projection), and its gradients agree with central
  differences.
* The triangulation's tables pair each face with a face of the neighbour that
  has the same endpoints in reverse order (modulo the period).
* A uniform state in uniform motion is an exact solution: the right-hand side
  vanishes on a jittered periodic triangulation, and with horizontal slip
  walls for a horizontal flow.  A uniform rainy state at rest has the
  pointwise microphysics source as its only tendency, equal to the box
  reference's.
* The face flux along e_x and e_z is the box reference's Lax-Friedrichs flux
  (wave speed with the rain's fall speed), and it is antisymmetric under
  swapping the sides and the normal for any normal.
* Mass, momentum (g = 0) and energy are conserved to rounding.
* The saturated cloudy contact: the tendency of its projection converges to
  that of the exact solution at order ~k, and the translated contact at order
  ~k+1 (Section 4.1 reports order k+1 for smooth moist flow).
"""
import math

import numpy as np
import pytest

import oracle as O
from exact import moist_contact_at, tri_conservative, tri_l2
from paper_2305_13847_amd import synth

PER, WALL = synth.PERIODIC, synth.WALL


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_volume_rule_is_exact_to_degree_2k_plus_1(k):
    rs, w = O.tri_rule(k)
    assert len(w) == (k + 1) * (k + 2) and np.all(w > 0)
    assert np.all(rs >= 0) and np.all(rs.sum(axis=1) <= 1)
    for a in range(2 * k + 2):
        for b in range(2 * k + 2 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = float(np.sum(w * rs[:, 0] ** a * rs[:, 1] ** b))
            assert abs(got - exact) <= 1e-14 * exact + 1e-16, (a, b, got, exact)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_basis_orthonormal_and_spans_Pk(k):
    rs, w = O.tri_rule(k)
    psi, _, _ = O.tri_basis(k, rs)
    assert psi.shape[1] == (k + 1) * (k + 2) // 2
    G = (psi * w[:, None]).T @ psi
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13
    rng = np.random.default_rng(k)
    pts = rng.uniform(0, 1, size=(40, 2))
    pts = pts[pts.sum(axis=1) <= 1]
    phi_pts, _, _ = O.tri_basis(k, pts)
    for a in range(k + 1):
        for b in range(k + 1 - a):
            f = rs[:, 0] ** a * rs[:, 1] ** b
            c = psi.T @ (w * f)
            assert np.abs(phi_pts @ c - pts[:, 0] ** a * pts[:, 1] ** b).max() < 1e-12, (a, b)
    # nothing of degree k+1 is reproduced
    f = rs[:, 0] ** (k + 1)
    c = psi.T @ (w * f)
    assert np.abs(phi_pts @ c - pts[:, 0] ** (k + 1)).max() > 1e-4


def test_basis_gradients_match_differences():
    k, eps = 4, 1e-6
    rng = np.random.default_rng(7)
    pts = rng.uniform(0.05, 0.45, size=(12, 2))
    _, dr, ds = O.tri_basis(k, pts)
    pr, _, _ = O.tri_basis(k, pts + [eps, 0.0])
    mr, _, _ = O.tri_basis(k, pts - [eps, 0.0])
    ps, _, _ = O.tri_basis(k, pts + [0.0, eps])
    ms, _, _ = O.tri_basis(k, pts - [0.0, eps])
    assert np.abs((pr - mr) / (2 * eps) - dr).max() < 1e-6
    assert np.abs((ps - ms) / (2 * eps) - ds).max() < 1e-6


def test_face_flux_matches_the_box_flux_on_axes():
    mesh = synth.tri_mesh((2, 2), (0.0, 0.0), (10.0, 10.0), (PER, PER), 2)
    P0 = O.default_params()
    f = tri_conservative(1.0, O.rho_vs(P0, 285.0), 2e-3, 1e-3, 285.0, (3.0, -2.0), rain=True)
    nzq = mesh.nzq
    bg = dict(rho_d=np.full(nzq, f[0]), rho_m=np.full(nzq, f[1]), rho_r=np.full(nzq, f[2]), E=np.full(nzq, f[5]))
    P = O.default_params(g=0.0, rain=1, vr_const=6.0)
    o = O.TriOracle(mesh, P, 6, bg)
    box = synth.Mesh(2, [1, 1], [0.0, 0.0], [10.0, 10.0], [PER, PER], 1)
    ob = O.Oracle(box, P, 6, {key: np.full(box.nzq, bg[key][0]) for key in bg})
    rng = np.random.default_rng(3)
    scale = np.array([1e-3, 1e-4, 2e-4, 1.0, 1.0, 300.0])
    for _ in range(4):
        Um, Up = rng.standard_normal(6) * scale, rng.standard_normal(6) * scale
        for j, n in enumerate(([1.0, 0.0], [0.0, 1.0])):
            Ft = o.face(Um, Up, 5.0, n)
            Fb = ob.face(Um, 0, Up, 0, j)
            assert np.allclose(Ft, Fb, rtol=1e-12, atol=1e-9), (j, Ft, Fb)
        th = rng.uniform(0, 2 * np.pi)
        n = np.array([np.cos(th), np.sin(th)])
        assert np.allclose(o.face(Um, Up, 5.0, n), -o.face(Up, Um, 5.0, -n), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("bc", [(PER, PER), (PER, WALL)])
def test_mesh_tables_pair_reversed_edges(bc):
    m = synth.tri_mesh((5, 4), (0.0, 0.0), (3.0, 2.0), bc, 2, jitter=0.2, seed=2)
    L = np.array([3.0, 2.0])
    xy = m.xy
    det = (xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1]) \
        - (xy[:, 2, 0] - xy[:, 0, 0]) * (xy[:, 1, 1] - xy[:, 0, 1])
    assert np.all(det > 0)
    walls = 0
    for e in range(m.ne):
        for f in range(3):
            e2, f2 = m.nb[e, f], m.nbf[e, f]
            if e2 < 0:
                walls += 1
                z = xy[e, [f, (f + 1) % 3], 1]
                assert np.allclose(z, 0.0) or np.allclose(z, 2.0)
                continue
            assert m.nb[e2, f2] == e and m.nbf[e2, f2] == f
            a, b = xy[e, f], xy[e, (f + 1) % 3]
            a2, b2 = xy[e2, f2], xy[e2, (f2 + 1) % 3]
            s = np.round((a - b2) / L) * L            # periodic shift, if any
            assert np.allclose(a - s, b2) and np.allclose(b - s, a2)
    assert walls == (0 if bc[1] == PER else 2 * 5)


def _uniform_case(mesh, u, rain=False, T0=285.0, cloud=2e-3, rr=0.0, shift=1000.0, g=0.0, vr=0.0):
    P0 = O.default_params()
    rvs = O.rho_vs(P0, T0)
    f = tri_conservative(1.0, rvs, cloud, rr, T0, u, rain)
    nzq = mesh.nzq
    bg = dict(rho_d=np.full(nzq, f[0]), rho_m=np.full(nzq, f[1]),
              rho_r=np.full(nzq, f[2] if rain else 0.0), E=np.full(nzq, f[-1] - shift))
    nv = len(f)

    def ps(xz):
        sh = xz.shape[:-1]
        vals = [0.0, 0.0] + ([0.0] if rain else []) + [f[-3], f[-2], shift]
        return np.stack([np.full(sh, v) for v in vals])
    P = O.default_params(g=g, rain=int(rain), vr_const=vr)
    o = O.TriOracle(mesh, P, nv, bg)
    return o, o.state(ps), f


@pytest.mark.parametrize("k", [1, 3])
def test_uniform_flow_is_steady(k):
    mesh = synth.tri_mesh((5, 4), (0.0, 0.0), (10.0, 8.0), (PER, PER), k, jitter=0.25, seed=3)
    o, C, _ = _uniform_case(mesh, (30.0, -12.0))
    dC = o.rhs(C)
    # the pressure flux alone is ~1e5 / h: the residual is rounding
    assert np.abs(dC).max() < 1e-12 * 1e5 / 2.0, np.abs(dC).max()


def test_horizontal_flow_between_walls_is_steady():
    mesh = synth.tri_mesh((5, 4), (0.0, 0.0), (10.0, 8.0), (PER, WALL), 3, jitter=0.25, seed=4)
    o, C, _ = _uniform_case(mesh, (30.0, 0.0))
    assert np.abs(o.rhs(C)).max() < 1e-12 * 1e5 / 2.0


def test_uniform_rain_has_only_the_pointwise_source():
    mesh = synth.tri_mesh((3, 3), (0.0, 0.0), (10.0, 10.0), (PER, PER), 2, jitter=0.2, seed=5)
    # the state is the background itself: the pressure perturbation is rounding
    # of p ~ 1e5, and the only other flux is the rain's fall
    o, C, f = _uniform_case(mesh, (0.0, 0.0), rain=True, rr=5e-4, cloud=4e-3, vr=5.0, shift=0.0)
    dC = o.rhs(C)
    # the same state on the box reference: dU/dt = G at every node
    box = synth.Mesh(2, [1, 1], [0.0, 0.0], [10.0, 10.0], [PER, PER], 1)
    bgb = {key: np.full(box.nzq, o._bg[i][0]) for i, key in enumerate(("rho_d", "rho_m", "rho_r", "E"))}
    ob = O.Oracle(box, o.P, 6, bgb)
    U = np.zeros((6, 1, 4))
    for v in range(6):
        U[v] = o.eval(C[v:v + 1], np.array([[0.3, 0.3]]))[0, 0, 0]
    G = ob.rhs(U)[:, 0, 0]
    assert np.abs(G[[0, 3, 4]]).max() < 1e-9 * np.abs(G).max()
    # constant fields have coefficient value / psi_0 with psi_0 = sqrt(2) in mode 0 only
    rounding = 1e-15 * 1e5
    assert np.abs(dC[:, :, 1:]).max() < rounding
    want = G / math.sqrt(2.0)
    for v in range(6):
        assert np.allclose(dC[v, :, 0], want[v], rtol=1e-10, atol=rounding)


def _smooth_state(mesh, L, seed, u=(40.0, 25.0)):
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, size=4)

    def ps(xz):
        x, z = xz[..., 0] / L[0], xz[..., 1] / L[1]
        s1 = np.sin(2 * np.pi * x + ph[0]) * np.cos(2 * np.pi * z + ph[1])
        s2 = np.cos(2 * np.pi * (x + z) + ph[2])
        T = 285.0 + 3.0 * s1
        rv = np.array([O.rho_vs(O.default_params(), float(t)) for t in T.ravel()]).reshape(T.shape)
        rc = 2e-3 * (1.2 + s2)
        rd = (8e4 / T - rv * 461.51) / 287.05
        f = tri_conservative(rd, rv, rc, 0.0 * T, T, [u[0] * (1 + 0.1 * s2), u[1] * (1 - 0.1 * s1)])
        return np.stack([f[0] - 0.9, f[1] - 0.01, f[2], f[3], f[4] - 2.5e4])
    return ps


@pytest.mark.parametrize("bc", [(PER, PER), (PER, WALL)])
def test_conservation(bc):
    L = (10.0, 8.0)
    mesh = synth.tri_mesh((6, 5), (0.0, 0.0), L, bc, 3, jitter=0.2, seed=6)
    nzq = mesh.nzq
    bg = dict(rho_d=np.full(nzq, 0.9), rho_m=np.full(nzq, 0.01), rho_r=np.zeros(nzq), E=np.full(nzq, 2.5e4))
    o = O.TriOracle(mesh, O.default_params(g=0.0), 5, bg)
    C = o.state(_smooth_state(mesh, L, 1))
    dC = o.rhs(C)
    xy = mesh.xy
    det = (xy[:, 1, 0] - xy[:, 0, 0]) * (xy[:, 2, 1] - xy[:, 0, 1]) \
        - (xy[:, 2, 0] - xy[:, 0, 0]) * (xy[:, 1, 1] - xy[:, 0, 1])
    total = np.sum(det[None, :] * dC[:, :, 0], axis=1)
    scale = np.sum(det[None, :] * np.abs(dC[:, :, 0]), axis=1)
    conserved = [0, 1, 2, 4] + ([3] if bc[1] == PER else [])
    assert np.all(np.abs(total[conserved]) < 1e-12 * scale[conserved]), (total, scale)
    if bc[1] == WALL:
        # the walls push on the vertical momentum
        assert abs(total[3]) > 1e-6 * scale[3]


def _contact(k, n, t, lo=(0.0, 0.0), L=(10.0, 10.0), u0=(1000.0, 500.0)):
    mesh = synth.tri_mesh((n, n), lo, (lo[0] + L[0], lo[1] + L[1]), (PER, PER), k, jitter=0.15, seed=n)

    def ps(tt):
        def f(xz):
            X = [xz[..., 0], xz[..., 1]]
            rd, rv, rc, rr, T, u = moist_contact_at(X, lo, L, tt, u0=u0)
            return np.stack(tri_conservative(rd, rv, rc, rr, T, u))
        return f
    f0 = ps(0.0)(np.array([[0.5, 0.5]]))[:, 0]
    nzq = mesh.nzq
    bg = dict(rho_d=np.full(nzq, f0[0]), rho_m=np.full(nzq, f0[1]), rho_r=np.zeros(nzq), E=np.full(nzq, f0[4]))
    o = O.TriOracle(mesh, O.default_params(g=0.0), 5, bg)
    shift = np.array([f0[0], f0[1], 0.0, 0.0, f0[4]])[:, None, None]

    def coeffs(tt):
        vals = ps(tt)(o.points()) - np.array([f0[0], f0[1], 0.0, 0.0, f0[4]])[:, None, None]
        return o.project(vals)
    del shift
    return o, coeffs


@pytest.mark.parametrize("k", [2, 3])
def test_contact_tendency_is_consistent(k):
    errs = []
    for n in (4, 8):
        o, coeffs = _contact(k, n, 0.0)
        d = 1e-7
        want = (coeffs(d) - coeffs(-d)) / (2 * d)
        got = o.rhs(coeffs(0.0))
        errs.append(max(tri_l2(o, got - want)[v] / tri_l2(o, want)[v] for v in range(5)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > k - 0.5, (errs, rate)


@pytest.mark.parametrize("k,ns", [(1, (8, 16, 32)), (2, (8, 16, 32)), (3, (4, 8, 16))])
def test_moist_contact_order(k, ns):
    tend = 0.25 * 10.0 / 1118.0
    errs = []
    for n in ns:
        o, coeffs = _contact(k, n, tend)
        dt0 = 0.1 * (10.0 / n) / ((2 * k + 1) * (1118.0 + 360.0))
        nst = int(np.ceil(tend / dt0))
        C1, _ = o.rk(coeffs(0.0), tend / nst, nst)
        Ce = coeffs(tend)
        e, ref = tri_l2(o, C1 - Ce), tri_l2(o, Ce)
        errs.append(max(e[v] / ref[v] for v in range(5) if ref[v] > 0))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    overall = 0.5 * np.log2(errs[0] / errs[2])
    assert overall >= k + 1 - 0.3 and rates.min() >= k + 1 - 0.6, (errs, rates, overall)

