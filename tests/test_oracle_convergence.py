"""Pins of the reference by exact solutions: order of accuracy in space and time.

* A saturated cloudy contact (uniform p and u, varying T, vapour at saturation,
  varying cloud water) is translated exactly; advected faster than sound the
  Lax-Friedrichs flux is close to upwind and the error falls at order ~k+1
  (the paper reports order k+1 for smooth moist flow, Section 4.1).
* The dry isentropic vortex (moist system with rho_m = rho_r = 0 is the Euler
  system with gamma = 1 + R_d/c_vd) pins the pressure terms.
* A spatially uniform rainy state with g = 0 reduces the scheme to the 0-D ODE
  dU/dt = G(U); the RK step must converge at third order to scipy's solution.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as O
from exact import conservative, l2, moist_contact, periodic_mesh, vortex


def _run(f, k, n, tend, umax, L=10.0, cfl=0.2):
    mesh = periodic_mesh((n, n), k, L=L)
    P = O.default_params(g=0.0)
    U0, bg = conservative(mesh, *f(mesh, 0.0))
    Ue, _ = conservative(mesh, *f(mesh, tend), bg=bg)
    o = O.Oracle(mesh, P, 5, bg)
    dt0 = cfl * mesh.h[0] / ((2 * k + 1) * umax)
    ns = int(np.ceil(tend / dt0))
    U1, _ = o.rk(U0, tend / ns, ns)
    return max(l2(mesh, U1[v] - Ue[v]) / l2(mesh, Ue[v]) for v in range(5) if l2(mesh, Ue[v]) > 0)


@pytest.mark.parametrize("k,ns", [(1, (8, 16, 32)), (2, (16, 32, 64)), (3, (4, 8, 16)), (4, (4, 8, 16))])
def test_moist_contact_order(k, ns):
    # three levels: the rate over the two halvings is at least k + 1 - 0.3,
    # and neither halving alone falls below k + 1 - 0.6
    f = lambda m, t: moist_contact(m, t, u0=(1000.0, 500.0))
    e = [_run(f, k, n, 0.25 * 10.0 / 1118.0, 1118.0 + 360.0) for n in ns]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    overall = 0.5 * np.log2(e[0] / e[2])
    assert overall >= k + 1 - 0.3 and rates.min() >= k + 1 - 0.6, (e, rates, overall)


def test_vortex_order_q3():
    f = lambda m, t: vortex(m, t, u0=(2.0, 1.0), r0=1.0)
    tend = 0.25 * 10.0 / (2.24 * 316.0)
    e = [_run(f, 3, n, tend, 2.5 * 316 + 330) for n in (8, 16, 32)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert e[-1] < 2e-3 and rates[-1] > 3.3, (e, rates)


def test_vortex_converges_q2():
    f = lambda m, t: vortex(m, t, u0=(2.0, 1.0), r0=1.0)
    tend = 0.25 * 10.0 / (2.24 * 316.0)
    e = [_run(f, 2, n, tend, 2.5 * 316 + 330) for n in (8, 16, 32)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert rates[-1] > 2.1 and rates[-1] > rates[0], (e, rates)


@pytest.mark.parametrize("scheme,order", [(0, 3), (1, 3)])
def test_rk_order_on_microphysics_ode(scheme, order):
    mesh = periodic_mesh((1, 1), 1)
    P = O.default_params(rain=1, g=0.0)
    ones = np.ones((1, 4))
    T0 = 286.0
    rvs = O.rho_vs(P, T0)
    # saturated cloudy air with rain: autoconversion and accretion active
    U, bg = conservative(mesh, 1.05 * ones, rvs * ones, 4e-3 * ones, 5e-4 * ones, T0 * ones,
                         [0 * ones, 0 * ones], rain=True)
    o = O.Oracle(mesh, P, 6, bg)
    tend = 400.0

    def f(t, y):
        V = np.broadcast_to(y[:, None, None], U.shape).copy()
        return o.rhs(V)[:, 0, 0]
    ref = solve_ivp(f, (0, tend), U[:, 0, 0], method="DOP853", rtol=1e-13, atol=1e-16).y[:, -1]
    errs = []
    for nst in (10, 20, 40):
        U1, _ = o.rk(U, tend / nst, nst, scheme=scheme)
        errs.append(abs(U1[2, 0, 0] - ref[2]) / abs(ref[2] - U[2, 0, 0]))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert abs(rates[-1] - order) < 0.3, (errs, rates)
