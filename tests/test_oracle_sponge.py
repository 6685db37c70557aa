"""Pins of the reference's sponge layer (Section 3.6).

The blending function is checked at the points where its value is fixed:
- 0 below z_D and continuous there with zero slope;
- alpha/2 halfway up the layer;
- alpha at the top;
- increasing in between.

The end-of-step map is checked against properties of the paper's update:
- it leaves nodes below the layer untouched;
- with alpha = 1 at the top it sends the moist perturbations, the momentum
  and E' to the far field (0, 0, 0, 0) and puts the moist mass into rho_d';
- it keeps the total density of every node;
- it is linear;
- it leaves the background (zero perturbation) alone.

In the RK step the sponge closes the step. Total mass stays conserved over
several sponge steps. The tangent of a sponge step matches central finite
differences of the reference's own forward step.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_13847_amd import synth

ZD, ALPHA = 6.0e3, 0.4


def _case(rain=False):
    if rain:
        return synth.warm_rain_3d(n=(3, 3, 6), order=3, seed=2)
    return synth.moist_bubble(n=(8, 6), order=3, seed=1)


def _oracle(c, zD=ZD, alpha=ALPHA):
    P = O.default_params(g=c.g, rain=c.rain, vr_const=c.vr_const, sponge_zD=zD, sponge_alpha=alpha)
    return O.Oracle(c.mesh, P, c.nvars, c.bg)


def test_blending_function_fixed_points():
    c = _case()
    o = _oracle(c)
    zT = c.mesh.hi[c.mesh.dim - 1]
    for z in (0.0, 1e3, ZD - 1.0, ZD):
        assert o.sponge_delta(z) == 0.0
    assert o.sponge_delta(0.5 * (ZD + zT)) == pytest.approx(ALPHA / 2, rel=1e-15)
    assert o.sponge_delta(zT) == pytest.approx(ALPHA, rel=1e-15)
    zs = np.linspace(ZD, zT, 201)
    ds = np.array([o.sponge_delta(z) for z in zs])
    assert np.all(np.diff(ds) > 0)
    # C1 at z_D: delta(z_D + eps) = O(eps^2)
    for eps in (1.0, 0.1):
        assert o.sponge_delta(ZD + eps) < 1e-6 * eps


def test_nodes_below_the_layer_are_untouched():
    c = _case()
    o = _oracle(c)
    S = o.sponge(c.U)
    z = synth.node_coords(c.mesh)[-1]
    below = z < ZD
    assert np.array_equal(S[:, below], c.U[:, below])
    assert not np.array_equal(S[:, ~below], c.U[:, ~below])


def test_full_strength_at_the_top_reaches_the_far_field():
    c = _case(rain=True)
    o = _oracle(c, alpha=1.0)
    S = o.sponge(c.U)
    z = synth.node_coords(c.mesh)[-1]
    top = z == c.mesh.hi[-1]
    assert top.any()
    assert np.all(S[1:, top] == 0.0)                               # rho_m', rho_r', m, E'
    np.testing.assert_allclose(S[0, top], c.U[0, top] + c.U[1, top] + c.U[2, top], rtol=1e-15, atol=1e-18)


@pytest.mark.parametrize("rain", [False, True])
def test_total_density_of_every_node_is_kept(rain):
    c = _case(rain)
    o = _oracle(c)
    S = o.sponge(c.U)
    nm = 3 if rain else 2
    before, after = c.U[:nm].sum(axis=0), S[:nm].sum(axis=0)
    assert np.max(np.abs(after - before)) <= 1e-15 * np.max(np.abs(c.U[:nm]))
    # and what left the moist variables went into rho_d'
    moved = (c.U[1:nm] - S[1:nm]).sum(axis=0)
    np.testing.assert_allclose(S[0] - c.U[0], moved, rtol=1e-12, atol=1e-19)


def test_sponge_is_linear_and_keeps_the_background():
    c = _case(rain=True)
    o = _oracle(c)
    rng = np.random.default_rng(4)
    A, B = rng.standard_normal(c.U.shape), rng.standard_normal(c.U.shape)
    a, b = 0.7, -1.3
    np.testing.assert_allclose(o.sponge(a * A + b * B), a * o.sponge(A) + b * o.sponge(B), rtol=1e-13, atol=1e-13)
    Z = np.zeros_like(c.U)
    assert np.array_equal(o.sponge(Z), Z)
    # alpha = 0: the identity
    assert np.array_equal(_oracle(c, alpha=0.0).sponge(c.U), c.U)


@pytest.mark.parametrize("scheme", [0, 1])
def test_sponge_closes_the_step(scheme):
    c = _case()
    with_, _ = _oracle(c).rk(c.U, c.dt, 1, scheme=scheme)
    plain, _ = _oracle(c, alpha=0.0).rk(c.U, c.dt, 1, scheme=scheme)
    np.testing.assert_array_equal(with_, _oracle(c).sponge(plain))


def test_mass_is_conserved_over_sponge_steps():
    c = _case()                                   # walls top and bottom, no rain
    o = _oracle(c, alpha=0.8)
    m0 = o.mass(c.U)
    U, _ = o.rk(c.U, c.dt, 6)
    m1 = o.mass(U)
    tot0, tot1 = m0[0] + m0[1], m1[0] + m1[1]
    assert abs(tot1 - tot0) <= 1e-12 * max(abs(tot0), 1e-3)


def test_tangent_of_a_sponge_step_matches_finite_differences():
    c = _case()
    o = _oracle(c)
    U = c.U.copy()
    for i in range(c.mesh.dim):
        U[c.nvars - 1 - c.mesh.dim + i] += 3.0 + i     # keep |u_j| off its kink
    rng = np.random.default_rng(9)
    V = rng.standard_normal(U.shape) * np.array([1e-4, 1e-5] + [1e-2] * c.mesh.dim + [10.0])[:, None, None]
    _, JV = o.rk_jvp(U, V, c.dt, 1)
    h = 1e-4
    Up, _ = o.rk(U + h * V, c.dt, 1)
    Um, _ = o.rk(U - h * V, c.dt, 1)
    fd = (Up - Um) / (2 * h)
    for v in range(c.nvars):
        scale = np.max(np.abs(fd[v])) + 1e-300
        assert np.max(np.abs(JV[v] - fd[v])) <= 1e-6 * scale, v
