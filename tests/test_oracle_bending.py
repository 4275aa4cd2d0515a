"""Pins of the oracle's light-bending and time-delay primitives (Sect. 2.3,
Sect. 2.8.2) against quantities the oracle does not compute itself:

* the original radial integrals Eq. (12) and Eq. (15), evaluated with mpmath
  in the variable w = R_S / r (the oracle integrates the finite forms
  Eqs. 32 and 35 in x);
* the periastron construction of inward rays (the oracle uses Eq. 34 with
  the closed-form root Eq. 14; here the periastron is found numerically from
  the conserved impact parameter and both legs are integrated radially);
* closed forms and limits: zero deflection at alpha = 0, the straight-line
  limit u -> 0, rho(u, pi/2) = 1, the cubic that rho solves, the grazing
  impact parameter b_max = R / sqrt(1 - u);
* the inverse map round trip and d cos(alpha) / d cos(psi) by differences.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle

mp.mp.dps = 30


def psi_radial(u, a):
    """Eq. (12) with w = R_S/r: psi = int_0^u dw / sqrt(p^2 - w^2 + w^3),
    p = R_S / b = u sqrt(1-u) / sin(alpha)."""
    u = mp.mpf(u)
    a = mp.mpf(a)
    p2 = (u * mp.sqrt(1 - u) / mp.sin(a)) ** 2
    return mp.quad(lambda w: 1 / mp.sqrt(p2 - w * w + w ** 3), [0, u])


def psi_radial_grazing(u):
    """Eq. (12) at alpha = pi/2 with w = u - t^2 (integrand made regular)."""
    u = mp.mpf(u)
    return mp.quad(lambda t: 2 / mp.sqrt((2 * u - 3 * u * u) + t * t * (3 * u - 1) - t ** 4), [0, mp.sqrt(u)])


def periastron_w(u, a):
    """Root of p^2 - w^2 + w^3 on (u, 2/3) (the function decreases there), by
    bisection in 30-digit arithmetic."""
    u = mp.mpf(u)
    p2 = (u * mp.sqrt(1 - u) / mp.sin(mp.mpf(a))) ** 2
    lo, hi = u, mp.mpf(2) / 3
    for _ in range(110):
        mid = (lo + hi) / 2
        if p2 - mid * mid + mid ** 3 > 0:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2, p2


def psi_radial_inward(u, a):
    """Inward ray: from R down to the periastron and out to infinity at the
    same impact parameter: psi = 2 int_0^{w_p} - int_0^u."""
    wp, p2 = periastron_w(u, a)
    h = lambda t: 2 * t / mp.sqrt(abs(p2 - (wp - t * t) ** 2 + (wp - t * t) ** 3))
    g = lambda w: 1 / mp.sqrt(p2 - w * w + w ** 3)
    return 2 * mp.quad(h, [0, mp.sqrt(wp)]) - mp.quad(g, [0, mp.mpf(u)])


def tp_radial(u, a):
    """Eq. (15) in units of R with r = R_S/w."""
    u = mp.mpf(u)
    a = mp.mpf(a)
    bb = (mp.sin(a) / (u * mp.sqrt(1 - u))) ** 2
    f = lambda w: u / (w * w * (1 - w)) * (1 / mp.sqrt(1 - bb * w * w * (1 - w)) - 1)
    return mp.quad(f, [0, u])


def tp_radial_from(w0, p2):
    """c dt_p measured in units of R_S, from radius R_S/w0 outwards, for a ray
    with (R_S/b)^2 = p2 (Eq. 15 written for an arbitrary start radius).
    w = w0 - t^2 makes the turning-point endpoint regular."""
    def f(w):
        return 1 / (w * w * (1 - w)) * (mp.sqrt(p2 / abs(p2 - w * w + w ** 3)) - 1)
    return mp.quad(lambda t: 2 * t * f(w0 - t * t), [0, mp.sqrt(w0)])


@pytest.mark.parametrize("u", [0.2, 0.3446, 0.5, 0.56])
@pytest.mark.parametrize("a", [1e-3, 0.3, 1.0, 1.5, 1.5707, math.pi / 2 - 1e-7])
def test_psi_matches_radial_integral(u, a):
    assert oracle.psi(u, a) == pytest.approx(float(psi_radial(u, a)), rel=2e-13)


@pytest.mark.parametrize("u,deg", [(0.2, None), (0.3446, None), (0.5, None), (0.56, None)])
def test_psi_grazing(u, deg):
    assert oracle.psi(u, math.pi / 2) == pytest.approx(float(psi_radial_grazing(u)), rel=1e-13)


@pytest.mark.parametrize("u", [0.2, 0.3446, 0.5])
@pytest.mark.parametrize("a", [0.3, 1.0, 1.5, 1.5707])
def test_time_delay_matches_radial_integral(u, a):
    assert oracle.tp(u, a) == pytest.approx(float(tp_radial(u, a)), rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("u", [0.25, 0.34, 0.45])
@pytest.mark.parametrize("da", [0.01, 0.1, 0.2])
def test_inward_branch_matches_periastron_integral(u, da):
    a = math.pi / 2 + da
    if a >= oracle.alpha_capture(u):
        pytest.skip("captured ray")
    assert oracle.psi(u, a) == pytest.approx(float(psi_radial_inward(u, a)), rel=1e-12)


@pytest.mark.parametrize("u", [0.25, 0.34, 0.45])
@pytest.mark.parametrize("da", [0.01, 0.15])
def test_inward_delay_is_two_legs(u, da):
    """Eq. (17) read in time units: the periastron leg counts twice, the leg
    from R once (negative), each measured from its own radius; the oracle's
    c dt_p / R of the inward ray must equal that sum divided by R."""
    a = math.pi / 2 + da
    wp, p2 = periastron_w(u, a)
    legs = 2 * tp_radial_from(wp, p2) - tp_radial_from(mp.mpf(u), p2)   # units of R_S
    assert oracle.tp(u, a) == pytest.approx(float(legs * u), rel=1e-11)


def test_zero_deflection_and_straight_line_limit():
    for u in (0.1, 0.3, 0.5):
        assert oracle.psi(u, 0.0) == 0.0
        assert oracle.tp(u, 0.0) == 0.0
    u = 1e-10
    for a in (0.2, 0.9, 1.4, math.pi / 2):
        assert oracle.psi(u, a) == pytest.approx(a, rel=1e-9)
        # flat space: path difference to the sub-observer point is R (1 - cos alpha)
        assert oracle.tp(u, a) == pytest.approx(1 - math.cos(a), rel=1e-8, abs=1e-12)


@pytest.mark.parametrize("u", [0.2, 0.35, 0.5, 0.56])
def test_rho_closed_form(u):
    assert oracle.rho(u, math.pi / 2) == pytest.approx(1.0, abs=1e-15)
    for a in (1.6, 1.7, 1.8):
        if a >= oracle.alpha_capture(u):
            continue
        r = oracle.rho(u, a)
        k = math.sin(a) ** 2 / (1 - u)
        assert r ** 3 - k * r + k * u == pytest.approx(0.0, abs=1e-14)
        assert 1.5 * u < r < 1.0   # between photon sphere and the surface
        # periastron impact parameter equals the emission one: r_p/sqrt(1-u/r) = R sin a / sqrt(1-u)
        assert r / math.sqrt(1 - u / r) == pytest.approx(math.sin(a) / math.sqrt(1 - u), rel=1e-13)


@pytest.mark.parametrize("u", [0.2, 0.3446, 0.5])
def test_grazing_impact_parameter(u):
    """At alpha = pi/2 the ray is tangent: b_max = R/sqrt(1-u) is the turning
    point radius, i.e. p^2 = u^2 (1-u) is a root of p^2 - w^2 + w^3 at w = u."""
    p2 = (u * math.sqrt(1 - u)) ** 2
    assert p2 - u * u + u ** 3 == pytest.approx(0.0, abs=1e-16)
    # and the deflection's derivative there is finite and equals 2/(sqrt(1-u) q(0))
    q0 = 2 - u / (1 - u)
    assert oracle.dpsi_dalpha(u, math.pi / 2) == pytest.approx(2 / (math.sqrt(1 - u) * q0), rel=1e-14)


@pytest.mark.parametrize("u", [0.2, 0.3446, 0.5])
@pytest.mark.parametrize("a", [0.05, 0.7, 1.3, 1.56, math.pi / 2 + 0.05])
def test_dpsi_matches_numerical_derivative(u, a):
    if a > math.pi / 2:
        h = mp.mpf("1e-3")
        x = mp.mpf(a)
        d = (psi_radial_inward(u, x - h) - psi_radial_inward(u, x + h)
             + 8 * (psi_radial_inward(u, x + h / 2) - psi_radial_inward(u, x - h / 2))) / (6 * h)
    else:
        d = mp.diff(lambda t: psi_radial(u, t), mp.mpf(a))
    assert oracle.dpsi_dalpha(u, a) == pytest.approx(float(d), rel=1e-9)


def test_psi_monotone_and_smooth_through_grazing():
    u = 0.34
    amax = min(oracle.alpha_capture(u) - 1e-3, math.pi / 2 + 0.3)
    a = np.linspace(0, amax, 400)
    p = np.array([oracle.psi(u, x) for x in a])
    assert np.all(np.diff(p) > 0)
    # one-sided slopes at pi/2 agree (the two branches join smoothly)
    h = 1e-5
    left = (oracle.psi(u, math.pi / 2) - oracle.psi(u, math.pi / 2 - h)) / h
    right = (oracle.psi(u, math.pi / 2 + h) - oracle.psi(u, math.pi / 2)) / h
    assert left == pytest.approx(right, rel=1e-4)


def test_beloborodov_sanity_bound():
    """1 - cos(alpha) ~ (1 - cos(psi))(1 - u): an approximation (not a pin of
    digits), accurate to about 1e-3 at moderate angles."""
    u, a = 0.3446, 1.0
    p = oracle.psi(u, a)
    assert (1 - math.cos(a)) == pytest.approx((1 - math.cos(p)) * (1 - u), rel=3e-3)


@pytest.mark.parametrize("u", [0.25, 0.3446, 0.5])
def test_inverse_map_roundtrip_and_lensing_factor(u):
    amax = min(math.pi / 2 + 0.1, oracle.alpha_capture(u) - 1e-4)
    for a in (0.01, 0.5, 1.2, 1.55, math.pi / 2 + 0.05):
        if a > amax:
            continue
        ps = oracle.psi(u, a)
        out = oracle.invert(u, amax, ps)
        assert out is not None
        assert out[0] == pytest.approx(a, rel=1e-12)
        assert out[1] == pytest.approx(math.cos(a), abs=1e-13)
        # LF = d cos(alpha) / d cos(psi) by central differences of the inverse
        h = 1e-6
        ap = oracle.invert(u, amax, math.acos(math.cos(ps) + h))[1]
        am = oracle.invert(u, amax, math.acos(math.cos(ps) - h))[1]
        assert out[2] == pytest.approx((ap - am) / (2 * h), rel=1e-6)
        assert out[3] == pytest.approx(math.sin(a) / math.sin(ps), rel=1e-12)
    # beyond the last visible ray: no image
    assert oracle.invert(u, amax, oracle.psi(u, amax) + 1e-6) is None
    # sub-observer limit: LF -> 1 - u
    out = oracle.invert(u, amax, 1e-9)
    assert out[2] == pytest.approx(1 - u, rel=1e-12)
    h = 1e-4
    ps = h
    out = oracle.invert(u, amax, ps)
    assert out[2] == pytest.approx(1 - u, rel=1e-6)
