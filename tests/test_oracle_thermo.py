"""Pins of the reference's thermodynamics and implicit-condensation split.

* e_s(T_ref) = e_ref and the Clausius-Clapeyron identity with a linear latent
  heat (Section 2.1);
* the split inverts the explicit forward map (T, rho_d, rho_v, rho_c) -> rho e
  on both branches (Section 2.2), agrees with brute-force bisection, and its
  tangent agrees with finite differences;
* the wave speed reduces to the dry and pure-vapour sound speeds.
"""
import math

import numpy as np
import pytest

import oracle as O

P = O.default_params()


def test_constants_table():
    # appendix table
    assert (P.cl, P.cpd, P.cpv, P.cvd, P.cvv) == (4218, 1005, 1850, 718, 1390)
    assert (P.eref, P.Lref, P.Rd, P.Rv, P.Tref, P.pref) == (610.7, 2.835e6, 287.05, 461.51, 273.15, 1e5)


def test_esat_reference_point():
    assert O.esat(P, P.Tref) == pytest.approx(P.eref, rel=1e-15)


@pytest.mark.parametrize("T", [220.0, 250.0, 273.15, 290.0, 310.0, 330.0])
def test_clausius_clapeyron(T):
    # d ln e_s / dT = L(T) / (R_v T^2) with L(T) = L_ref + (c_pv - c_l)(T - T_ref)
    h = 1e-3
    num = (math.log(O.esat(P, T + h)) - math.log(O.esat(P, T - h))) / (2 * h)
    L = P.Lref + (P.cpv - P.cl) * (T - P.Tref)
    assert num == pytest.approx(L / (P.Rv * T * T), rel=1e-8)


def test_rho_vs_is_vapour_eos():
    for T in (250.0, 300.0):
        assert O.rho_vs(P, T) == pytest.approx(O.esat(P, T) / (P.Rv * T), rel=1e-15)


def forward(rd, rm, rr, T):
    """Explicit forward map: temperature and densities -> rho e (energy relation)."""
    rv = min(O.rho_vs(P, T), rm)
    rc = rm - rv
    return (P.cvd * rd + P.cvv * rv + P.cl * (rc + rr)) * (T - P.Tref) + rv * (P.Lref - P.Rv * P.Tref), rv


def test_split_round_trip_random():
    rng = np.random.default_rng(11)
    nsat = 0
    worst = 0.0
    for _ in range(3000):
        T = rng.uniform(215.0, 320.0)
        rd = rng.uniform(0.3, 1.3)
        rvs = O.rho_vs(P, T)
        rm = rvs * rng.uniform(0.2, 1.8)
        rr = rng.choice([0.0, rng.uniform(0.0, 3e-3)])
        re, rv = forward(rd, rm, rr, T)
        T2, rv2, rc2, it = O.split(P, rd, rm, rr, re)
        assert it >= 0
        worst = max(worst, abs(T2 - T) / T)
        assert rv2 == pytest.approx(rv, rel=1e-12, abs=1e-18)
        assert rc2 == pytest.approx(rm - rv, abs=1e-14)
        nsat += rm > rvs
    assert worst < 1e-13
    assert 500 < nsat < 2500


def bisect_root(rd, rm, rr, re):
    """Brute force: bisection on the monotone map T -> rho e."""
    lo, hi = 100.0, 500.0
    g = lambda T: forward(rd, rm, rr, T)[0] - re
    assert g(lo) < 0 < g(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) < 0:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-13:
            break
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("case", range(12))
def test_split_matches_bisection(case):
    rng = np.random.default_rng(100 + case)
    rd = rng.uniform(0.4, 1.2)
    rm = rng.uniform(0.002, 0.04)
    rr = rng.uniform(0.0, 2e-3) if case % 2 else 0.0
    re = forward(rd, rm, rr, rng.uniform(250.0, 305.0))[0] + rng.normal(0, 50.0)
    Tb = bisect_root(rd, rm, rr, re)
    T, rv, rc, it = O.split(P, rd, rm, rr, re)
    assert T == pytest.approx(Tb, abs=1e-10)
    assert rv <= rm + 1e-18
    assert rc >= -1e-18


def test_split_monotone_and_unique():
    rd, rm, rr = 1.0, 0.03, 0.0
    Ts = np.linspace(230.0, 320.0, 2001)
    re = np.array([forward(rd, rm, rr, T)[0] for T in Ts])
    assert np.all(np.diff(re) > 0)


def test_split_branches():
    # unsaturated: no cloud; saturated: vapour at saturation
    rd = 1.0
    T = 290.0
    rvs = O.rho_vs(P, T)
    re, _ = forward(rd, 0.5 * rvs, 0.0, T)
    T2, rv, rc, it = O.split(P, rd, 0.5 * rvs, 0.0, re)
    assert it == 0 and rc == 0.0 and rv == 0.5 * rvs
    re, _ = forward(rd, 1.5 * rvs, 0.0, T)
    T2, rv, rc, it = O.split(P, rd, 1.5 * rvs, 0.0, re)
    assert it > 0 and rc == pytest.approx(0.5 * rvs, rel=1e-12)


def test_split_rejects_nonpositive_temperature():
    T, rv, rc, it = O.split(P, 1.0, 0.01, 0.0, -1e6)
    assert it == -1


@pytest.mark.parametrize("sat", [False, True])
def test_split_tangent_vs_finite_difference(sat):
    rng = np.random.default_rng(7 + sat)
    rd, T0 = 1.05, 288.0
    rvs = O.rho_vs(P, T0)
    rm = rvs * (1.3 if sat else 0.7)
    rr = 1e-3
    re = forward(rd, rm, rr, T0)[0]
    x = np.array([rd, rm, rr, re])
    for _ in range(4):
        dx = rng.standard_normal(4) * np.array([1e-2, 1e-3, 1e-4, 1e2])
        T, dT, rv, drv = O.split_jvp(P, x, dx)
        h = 1e-4
        Tp, rvp, _, _ = O.split(P, *(x + h * dx))
        Tm, rvm, _, _ = O.split(P, *(x - h * dx))
        assert dT == pytest.approx((Tp - Tm) / (2 * h), rel=1e-6, abs=1e-12)
        assert drv == pytest.approx((rvp - rvm) / (2 * h), rel=1e-6, abs=1e-15)
