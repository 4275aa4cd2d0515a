"""Pins of the oracle's star shape, surface gravity, radial delay terms and
response fold against values fixed outside the oracle (Sects. 2.2, 2.3,
2.8.4).

* shape and gravity coefficients: the oracle's o2 and g(theta)/g0 sampled
  over many stars and colatitudes and regressed onto the monomials of the
  paper's relations; the recovered coefficients must equal the printed ones
  (``tests/golden/star_shape_coefficients.json``, Sect. 2.2) to rounding,
  and the fit must leave no residual (no missing or extra term);
* spot values of the two benchmark stars (Obar, o2, u range, log g
  range over a pole-to-pole band, equatorial speed, largest surface tilt),
  computed independently of the oracle and quoted at their printed rounding;
* oblate radial delay Eq. (delta_t_oblate): the coordinate light-travel
  distance of a radial photon, integral of dr / (1 - R_S / r) from R to R_e,
  by mpmath quadrature;
* total delay of a ray (Eqs. tp_direct, delta_t_oblate, tot_time_delay):
  the light-travel time along the Schwarzschild null geodesic integrated
  directly (both legs of an inward ray through its periastron, found as the
  root of the turning-point condition), relative to a radial photon from
  R_e;
* response fold (Sect. 2.8.4): counts = T_exp / P (F_t * exp(-N_H sigma)) @
  RSP with a random non-square RSP, against numpy.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
import synthetic as syn

GOLD = os.path.join(os.path.dirname(__file__), "golden", "star_shape_coefficients.json")


def band_spec(n_rings=400, mode=syn.MODE_OS):
    """One cap centred on the equator with radius pi/2: rings from pole to pole."""
    return dict(mode=mode, intensity=0, n_spots=1, shape=[0, 0], n_rings=[n_rings, n_rings],
                n_phi=[4, 4], shape_a=[0.0, 0.0], shape_b=[0.0, 0.0], n_fp=16, n_phase=4,
                energy=syn.logspace(0.3, 2.0, 4), t_exp=1.0, sigma=np.zeros(4), rsp=np.eye(4))


def band_params(M, Re, nu):
    return syn.params_vector(M, Re, 1.0, 0.0, 1.0, nu, 150.0, math.pi / 2, math.pi / 2, 6.0)


def star_samples():
    """(x, Obar, o2, theta, g/g0) over a grid of stars and a pole-to-pole band."""
    rows = []
    spec = band_spec(n_rings=24)
    for M in (1.0, 1.4, 1.9, 2.3):
        for Re in (9.0, 11.5, 14.0, 16.0):
            for nu in (150.0, 350.0, 550.0, 700.0):
                p = band_params(M, Re, nu)
                if syn.compactness(p)[0] > 0.3:
                    continue
                st = oracle.star(spec, p)
                for r in oracle.rings(spec, p, 0):
                    rows.append((st.x, st.Obar, st.o2, r.theta, 10.0 ** r.logg / st.g0))
    return np.array(rows)


def test_o2_coefficients_recovered():
    gold = json.load(open(GOLD))["o2_over_Obar2"]
    s = star_samples()
    x, Ob, o2 = s[:, 0], s[:, 1], s[:, 2]
    A = np.stack([np.ones_like(x), x], axis=1)
    coef, *_ = np.linalg.lstsq(A, o2 / Ob ** 2, rcond=None)
    assert coef[0] == pytest.approx(gold["1"], abs=1e-9)
    assert coef[1] == pytest.approx(gold["x"], abs=1e-9)
    assert np.max(np.abs(A @ coef - o2 / Ob ** 2)) < 1e-12


def test_gravity_coefficients_recovered():
    """Regression of g/g0 - 1 onto the monomials of the gravity relation.
    A coefficient of the oracle that differs from the printed one in its
    third significant digit moves the recovered value by >= 1e-3 (checked
    to 1e-7 here)."""
    g = json.load(open(GOLD))["gravity"]
    s = star_samples()
    x, Ob, th, ratio = s[:, 0], s[:, 1], s[:, 3], s[:, 4]
    O2, O4, O6 = Ob ** 2, Ob ** 4, Ob ** 6
    s2, c2, ac = np.sin(th) ** 2, np.cos(th) ** 2, np.abs(np.cos(th))
    cols, expect = [], []
    for ang, w in (("sin2", s2), ("cos2", c2)):
        for key, mono in (("O2", O2), ("O2*x", O2 * x), ("O4*x", O4 * x), ("O4*x2", O4 * x * x),
                          ("O6*x", O6 * x)):
            cols.append(w * mono)
            e = g[ang][key]
            if ang == "cos2" and key in g["cos2_minus"]:
                e -= g["cos2_minus"][key]
            expect.append(e)
    for key, mono in (("O4*x", O4 * x), ("O4*x2", O4 * x * x)):
        cols.append(ac * mono)
        expect.append(g["abscos"][key])
    A = np.stack(cols, axis=1)
    coef, *_ = np.linalg.lstsq(A, ratio - 1.0, rcond=None)
    np.testing.assert_allclose(coef, np.array(expect), rtol=0, atol=1e-7)
    assert np.max(np.abs(A @ coef - (ratio - 1.0))) < 1e-12


@pytest.mark.parametrize("cfg, want", [
    (syn.config1, dict(Obar=(0.3865, 5e-5), o2=(-0.0923, 5e-5), u=((0.3308, 0.3644), 5e-5),
                       logg=((14.115, 14.218), 5e-4), beta_eq=(0.192, 5e-4), eta_deg=(6.8, 0.05))),
    (syn.config2, dict(Obar=(0.297, 5e-4), o2=(-0.0441, 5e-5), u=((0.56, 0.586), 5e-4),
                       logg=((14.46, 14.51), 5e-3), beta_eq=(0.237, 5e-4), eta_deg=None)),
])
def test_benchmark_star_values(cfg, want):
    """The two benchmark stars' shape, gravity and speed at the rounding the
    values were quoted with (independent evaluation of Sect. 2.2)."""
    _, p = cfg(n_cells=8)
    q = band_params(p[0], p[1], p[5])
    spec = band_spec(n_rings=4000)
    st = oracle.star(spec, q)
    rg = oracle.rings(spec, q, 0)
    u = np.array([r.u for r in rg])
    lg = np.array([r.logg for r in rg])
    beta = np.array([r.beta for r in rg])
    eta = np.degrees(np.abs(np.arctan([r.f for r in rg])))
    assert st.Obar == pytest.approx(want["Obar"][0], abs=want["Obar"][1])
    assert st.o2 == pytest.approx(want["o2"][0], abs=want["o2"][1])
    (ulo, uhi), tol = want["u"]
    assert u.min() == pytest.approx(ulo, abs=tol) and u.max() == pytest.approx(uhi, abs=tol)
    (glo, ghi), tol = want["logg"]
    assert lg.min() == pytest.approx(glo, abs=tol) and lg.max() == pytest.approx(ghi, abs=tol)
    # gravity is lowest at the equator and highest at the poles
    assert np.argmin(lg) in (len(rg) // 2 - 1, len(rg) // 2)
    assert beta.max() == pytest.approx(want["beta_eq"][0], abs=want["beta_eq"][1])
    if want["eta_deg"]:
        assert eta.max() == pytest.approx(want["eta_deg"][0], abs=want["eta_deg"][1])


# ------------------------------------------------------------------ delays
def _star_for_delay(M, Re, nu):
    spec = band_spec(n_rings=8)
    p = band_params(M, Re, nu)
    return spec, p, oracle.star(spec, p)


@pytest.mark.parametrize("M, Re, nu", [(1.4, 12.5, 600.0), (2.0, 10.5, 600.0), (1.0, 15.0, 400.0)])
def test_oblate_radial_delay_quadrature(M, Re, nu):
    spec, p, st = _star_for_delay(M, Re, nu)
    mp.mp.dps = 30
    for frac in (1.0, 0.97, 0.9, 0.8):
        R = st.Re * frac
        want = mp.quad(lambda r: 1 / (1 - st.Rs / r), [R, st.Re]) if frac < 1 else mp.mpf(0)
        got = oracle.cdt_oblate(spec, p, R)
        assert abs(got - float(want)) <= 1e-11 * st.Re


def geodesic_delay(Rs, Re, R, alpha):
    """c dt of a photon emitted at radius R with angle alpha to the radial
    direction, relative to a radial photon emitted at R_e, from the null
    geodesic: c dt/dr = 1 / ((1 - R_S/r) sqrt(1 - (b/r)^2 (1 - R_S/r))),
    b = R sin(alpha) / sqrt(1 - R_S/R).  Inward rays (alpha > pi/2) run in
    to the periastron R_p (root of r^3 - b^2 (r - R_S) between the photon
    sphere 1.5 R_S and R) and back out.  Lengths in units of R inside."""
    mp.mp.dps = 30
    us, ue, a = mp.mpf(Rs) / mp.mpf(R), mp.mpf(Re) / mp.mpf(R), mp.mpf(alpha)
    b = mp.sin(a) / mp.sqrt(1 - us)
    f = lambda y: 1 / (1 - us / y)
    g = lambda y: f(y) / mp.sqrt(1 - (b / y) ** 2 * (1 - us / y))
    tail = mp.quad(lambda y: g(y) - f(y), [ue, 4 * ue, mp.inf])
    if a <= mp.pi / 2:
        return R, float(R * (tail + (mp.quad(g, [1, ue]) if ue > 1 else 0)))
    h = lambda y: y ** 3 - b * b * (y - us)
    lo, hi = mp.mpf(1.5) * us, mp.mpf(1)       # h(lo) < 0 < h(hi) for an escaping inward ray
    assert h(lo) < 0 < h(hi)
    for _ in range(120):
        mid = (lo + hi) / 2
        lo, hi = (mid, hi) if h(mid) < 0 else (lo, mid)
    yp = (lo + hi) / 2
    # near the turning point 1 - (b/y)^2 (1 - us/y) = (y - yp) q(y) / y^3 with
    # q(y) = y^2 + yp y + yp^2 - b^2 > 0; y = yp + t^2 removes the square-root
    # singularity of each leg
    q = lambda y: y * y + yp * y + yp * yp - b * b
    leg = lambda Y: mp.quad(lambda t: 2 * f(yp + t * t) * (yp + t * t) ** 1.5 / mp.sqrt(q(yp + t * t)),
                            [0, mp.sqrt(Y - yp)])
    legs = leg(1) + leg(ue)
    return float(R * yp), float(R * (legs + tail))


@pytest.mark.parametrize("M, Re, nu", [(1.4, 12.5, 600.0), (2.0, 10.5, 600.0)])
@pytest.mark.parametrize("frac_R", [1.0, 0.93])
def test_total_delay_geodesic(M, Re, nu, frac_R):
    """orc_total_delay (outgoing: Eq. tp_direct + Eq. delta_t_oblate;
    inward: Eq. tot_time_delay with the periastron leg) against the delay
    integrated along the geodesic itself."""
    spec, p, st = _star_for_delay(M, Re, nu)
    R = st.Re * frac_R
    u = st.Rs / R
    acap = oracle.alpha_capture(u)
    for alpha in (0.2, 1.0, 1.5, math.pi / 2 + 0.03, math.pi / 2 + 0.12, min(math.pi / 2 + 0.3, acap - 0.05)):
        Rp, want = geodesic_delay(st.Rs, st.Re, R, alpha)
        got = oracle.total_delay(spec, p, R, u, alpha) * R
        assert abs(got - want) <= 2e-9 * R, (alpha, got, want)
        if alpha > math.pi / 2:
            # the periastron of the formula (rho R) is the geodesic's turning point
            assert oracle.rho(u, alpha) * R == pytest.approx(Rp, rel=1e-12)


def test_inward_oblate_term_against_quadrature():
    """The oblate part of Eq. (tot_time_delay), 2 delta_t(R_p) - delta_t(R),
    on its own: total delay minus the spherical part, against quadrature of
    the radial travel distances of both legs."""
    spec, p, st = _star_for_delay(1.4, 12.5, 600.0)
    R = st.Re * 0.92
    u = st.Rs / R
    mp.mp.dps = 30
    for alpha in (math.pi / 2 + 0.05, math.pi / 2 + 0.2):
        Rp = oracle.rho(u, alpha) * R
        f = lambda r: 1 / (1 - st.Rs / r)
        want = 2 * mp.quad(f, [Rp, st.Re]) - mp.quad(f, [R, st.Re])
        got = (oracle.total_delay(spec, p, R, u, alpha) - oracle.tp(u, alpha)) * R
        assert abs(got - float(want)) <= 1e-10 * R


# -------------------------------------------------------------------- fold
def test_fold_general_response():
    """counts[k, c] = T_exp / P sum_e F_t[k, e] exp(-N_H sigma_e) RSP[e, c]
    with a random non-square RSP (E != C, no symmetry): a transposed index
    or a misplaced factor fails."""
    spec, p = syn.config1(n_cells=6, n_phase=7, n_energy=12)
    rng = np.random.default_rng(5)
    spec["rsp"] = rng.uniform(0.0, 50.0, size=(12, 17))
    spec["sigma"] = rng.uniform(0.5e-22, 3e-22, size=12)
    p[4] = 3.5
    ft, cnt, _ = oracle.forward(spec, p)
    assert cnt.shape == (7, 17)
    att = np.exp(-p[4] * 1e20 * spec["sigma"])
    want = (ft * att[None, :]) @ spec["rsp"] * (spec["t_exp"] / 7)
    np.testing.assert_allclose(cnt, want, rtol=1e-13, atol=0)
    # reading the response as [C][E] (a transposed index) gives other counts
    flat = spec["rsp"].ravel()
    wrong = np.array([[sum(ft[k, e] * att[e] * flat[c * 12 + e] for e in range(12)) for c in range(12)]
                      for k in range(7)]) * (spec["t_exp"] / 7)
    assert np.max(np.abs(wrong - cnt[:, :12]) / np.abs(cnt[:, :12])) > 1e-2
