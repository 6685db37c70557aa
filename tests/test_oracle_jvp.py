"""Pins of the reference's exact directional derivatives (forward mode).

The tangent of the right-hand side and of several RK steps must agree with
central finite differences of the reference itself; the split's tangent uses
the implicit-function derivative of the saturation system.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_13847_amd import synth


def _dirn(rng, U, scale):
    V = rng.standard_normal(U.shape)
    return V * scale[:, None, None]


@pytest.mark.parametrize("which", ["bubble", "rain3d"])
def test_rhs_jvp_vs_finite_difference(which):
    if which == "bubble":
        c = synth.moist_bubble(n=(5, 4), order=3, seed=3)
        scale = np.array([1e-4, 1e-5, 1e-2, 1e-2, 10.0])
    else:
        c = synth.warm_rain_3d(n=(3, 3, 3), order=2, seed=4)
        # rain bounded away from zero keeps the fractional powers smooth
        c.U[2] = np.abs(c.U[2]) + 2e-4
        # and saturated everywhere with a margin: off the split's kink
        c.U[1] += 0.5 * c.bg["rho_m"][synth.height_index(c.mesh)]
        scale = np.array([1e-4, 1e-5, 1e-6, 1e-2, 1e-2, 1e-2, 10.0])
    # a mean wind keeps every |u_j| away from its kink at zero
    for i in range(c.mesh.dim):
        c.U[c.nvars - 1 - c.mesh.dim + i] += 3.0 + i
    o = O.Oracle.for_case(c)
    rng = np.random.default_rng(9)
    V = _dirn(rng, c.U, scale)
    R0, JV = o.rhs_jvp(c.U, V)
    assert np.array_equal(R0, o.rhs(c.U))
    # nearly tied face maxima are kinks: a small step keeps FD off them
    h = 1e-4
    fd = (o.rhs(c.U + h * V) - o.rhs(c.U - h * V)) / (2 * h)
    for v in range(c.nvars):
        den = np.abs(fd[v]).max()
        assert np.abs(JV[v] - fd[v]).max() <= 1e-6 * den + 1e-30, v


def test_rk_jvp_vs_finite_difference():
    c = synth.moist_bubble(n=(5, 4), order=2, seed=4)
    c.U[2] += 3.0
    o = O.Oracle.for_case(c)
    rng = np.random.default_rng(10)
    V = _dirn(rng, c.U, np.array([1e-4, 1e-5, 1e-2, 1e-2, 10.0]))
    U1, V1 = o.rk_jvp(c.U, V, c.dt, 3)
    U1b, _ = o.rk(c.U, c.dt, 3)
    assert np.array_equal(U1, U1b)
    h = 1e-4
    fd = (o.rk(c.U + h * V, c.dt, 3)[0] - o.rk(c.U - h * V, c.dt, 3)[0]) / (2 * h)
    for v in range(c.nvars):
        assert np.abs(V1[v] - fd[v]).max() <= 1e-6 * np.abs(fd[v]).max()
