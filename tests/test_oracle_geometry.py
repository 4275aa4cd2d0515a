"""Pins of the oracle's star, ring and per-sample geometry (Sects. 2.1, 2.2,
2.4, 2.8.3).

* spot areas: the oracle's ring weights summed over a spot against a direct
  pixel integration of the Schwarzschild-induced area element of the surface
  r = R(theta) over the spot region (membership by angular distance);
* solid angle of a cap, 2 pi (1 - cos zeta);
* the angle formulas of the fine-phase trace (cos sigma Eq. 4, cos xi of
  Table 2, Doppler factor Eq. 19, aberration Eq. 20, redshift) recomputed
  from explicit 3D unit vectors;
* the invisible-segment fill (Eqs. 41-44);
* star quantities: S+D and non-rotating limits, equatorial symmetry.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as syn


def small_spec(mode=syn.MODE_OS, shape=(0, 1), n=32, nphi=32, n_fp=192, intensity=0, n_spots=2,
               shape_a=(0.0, 0.4), shape_b=(0.0, 0.0)):
    spec = dict(mode=mode, intensity=intensity, n_spots=n_spots, shape=list(shape), n_rings=[n, n],
                n_phi=[nphi, nphi], shape_a=list(shape_a), shape_b=list(shape_b), n_fp=n_fp, n_phase=8,
                energy=syn.logspace(0.3, 2.0, 4), t_exp=8.0, sigma=np.zeros(4), rsp=np.eye(4))
    return spec


def induced_area(params, mode, member, n_th=1500, n_ph=3000, th_range=(0.0, math.pi)):
    """Area of {member(theta, phi)} on the surface r = R(theta) with the
    Schwarzschild spatial metric dr^2/(1-R_S/r) + r^2 dOmega:
    dA = R sin(theta) sqrt(R^2 + R_theta^2 / (1 - R_S/R)) dtheta dphi."""
    GM = params[0] * syn.GM_SUN
    Re = params[1] * 1e5
    Rs = 2 * GM / syn.C_CGS ** 2
    x = GM / (syn.C_CGS ** 2 * Re)
    Ob = 2 * math.pi * params[5] * math.sqrt(Re ** 3 / GM)
    o2 = Ob ** 2 * (-0.788 + 1.030 * x) if mode == syn.MODE_OS else 0.0
    t0, t1 = th_range
    th = t0 + (np.arange(n_th) + 0.5) * (t1 - t0) / n_th
    ph = (np.arange(n_ph) + 0.5) * 2 * math.pi / n_ph - math.pi
    T, P = np.meshgrid(th, ph, indexing="ij")
    R = Re * (1 + o2 * np.cos(T) ** 2)
    Rt = -2 * Re * o2 * np.cos(T) * np.sin(T)
    dA = R * np.sin(T) * np.sqrt(R ** 2 + Rt ** 2 / (1 - Rs / R)) * ((t1 - t0) / n_th) * (2 * math.pi / n_ph)
    return float(np.sum(dA * member(T, P)))


def angdist(t1, p1, t2, p2):
    c = np.cos(t1) * np.cos(t2) + np.sin(t1) * np.sin(t2) * np.cos(p1 - p2)
    return np.arccos(np.clip(c, -1, 1))


@pytest.mark.parametrize("mode", [syn.MODE_SD, syn.MODE_OS])
def test_spot_area_cap_annulus(mode):
    spec = small_spec(mode=mode, n=128, nphi=64)
    p = syn.params_vector(1.4, 12.5, 1.0, 0.0, 1.0, 600.0, 150.0, 0.8, 0.3, 6.1, 2.2, 0.25, 6.0, 0.38)
    D = p[6] * syn.PC_CM
    for spot in (0, 1):
        rg = oracle.rings(spec, p, spot)
        a_rings = sum(r.w_cell * r.n_cells for r in rg) * D * D
        tc, z = p[8 + 4 * spot], p[9 + 4 * spot]
        if spot == 0:
            member = lambda T, P: angdist(T, P, tc, 0.0) <= z
        else:
            member = lambda T, P: (angdist(T, P, tc, 0.0) <= z) & (angdist(T, P, tc, 0.0) > 0.4 * z)
        a_pix = induced_area(p, mode, member, th_range=(max(0, tc - z), min(math.pi, tc + z)))
        assert a_rings == pytest.approx(a_pix, rel=2e-3)


def test_spot_area_pole_straddling_cap_and_crescent():
    spec = small_spec(shape=(0, 2), n=128, nphi=128, shape_a=(0.0, 0.8), shape_b=(0.0, 0.4))
    p = syn.params_vector(2.0, 12.5, 1.0, 0.0, 1.0, 600.0, 150.0, 0.3, 1.2, 6.0, math.radians(170), 0.3, 6.2, 0.3)
    D = p[6] * syn.PC_CM
    rg = oracle.rings(spec, p, 0)
    a_rings = sum(r.w_cell * r.n_cells for r in rg) * D * D
    a_pix = induced_area(p, syn.MODE_OS, lambda T, P: angdist(T, P, 0.3, 0.0) <= 1.2, th_range=(0.0, 1.5))
    assert a_rings == pytest.approx(a_pix, rel=2e-3)
    # crescent: the oracle masks cells whose centre lies in the mask cap;
    # compare the unmasked cell count x weight with the pixel area
    tc, z = p[12], p[13]
    tm, zm = tc - 0.4 * z, 0.8 * z      # spot in the south: the mask moves north
    member = lambda T, P: (angdist(T, P, tc, 0.0) <= z) & (angdist(T, P, tm, 0.0) > zm)
    a_pix = induced_area(p, syn.MODE_OS, member, n_th=1500, n_ph=4000, th_range=(tc - z, math.pi))
    rg = oracle.rings(spec, p, 1)
    tot = 0.0
    for r in rg:
        offs = -r.dphi_out + (np.arange(r.n_cells) + 0.5) * r.dphi_cell
        keep = angdist(r.theta, offs, tm, 0.0) > zm
        tot += r.w_cell * keep.sum()
    assert tot * D * D == pytest.approx(a_pix, rel=2e-2)


def test_cap_solid_angle_converges():
    spec = small_spec(mode=syn.MODE_SD, n=64, nphi=32)
    p = syn.params_vector(1.4, 12.0, 1.0, 0.0, 0.0, 0.0, 200.0, 1.1, 0.4, 6.0)
    rg = oracle.rings(spec, p, 0)
    omega = sum(r.dcos * r.dphi_cell * r.n_cells for r in rg)
    assert omega == pytest.approx(2 * math.pi * (1 - math.cos(0.4)), rel=1e-3)


def test_star_limits_and_symmetry():
    spec = small_spec(mode=syn.MODE_OS)
    p = syn.params_vector(1.4, 12.5, 1.0, 0.0, 1.0, 0.0, 150.0, 0.8, 0.3, 6.1, 2.2, 0.25, 6.0, 0.38)
    st = oracle.star(spec, p)
    assert st.o2 == 0.0 and st.Obar == 0.0
    rg = oracle.rings(spec, p, 0)
    for r in rg:
        assert r.R == pytest.approx(12.5e5, rel=1e-15)
        assert r.beta == 0.0 and r.f == 0.0
        assert 10 ** r.logg == pytest.approx(st.g0, rel=1e-13)
    p[5] = 600.0
    st = oracle.star(spec, p)
    assert st.x == pytest.approx(1.4 * syn.GM_SUN / (syn.C_CGS ** 2 * 12.5e5), rel=1e-15)
    assert st.Rs == pytest.approx(2 * st.x * st.Re, rel=1e-15)
    # mirrored spot: the ring geometry mirrors (theta -> pi - theta)
    q = p.copy()
    q[8] = math.pi - p[8]
    a = oracle.rings(spec, p, 0)
    b = oracle.rings(spec, q, 0)
    for ra, rb in zip(a, b[::-1]):
        assert rb.theta == pytest.approx(math.pi - ra.theta, abs=1e-14)
        assert rb.R == pytest.approx(ra.R, rel=1e-14)
        assert rb.logg == pytest.approx(ra.logg, abs=1e-13)
        assert rb.f == pytest.approx(-ra.f, rel=1e-12, abs=1e-18)
    # oblate: polar radius below the equatorial one, gravity higher at the pole
    assert st.o2 < 0


def vector_trace(spec, p, r, ifp):
    """Recompute one fine-phase sample from 3D unit vectors (observer in the
    x-z plane at inclination i, azimuth measured in the rotation direction)."""
    n_fp = spec["n_fp"]
    phi = 2 * math.pi * ifp / n_fp
    i = p[2]
    k = np.array([math.sin(i), 0.0, math.cos(i)])
    th = r.theta
    rh = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
    thh = np.array([math.cos(th) * math.cos(phi), math.cos(th) * math.sin(phi), -math.sin(th)])
    phh = np.array([-math.sin(phi), math.cos(phi), 0.0])
    cpsi = float(k @ rh)
    psi = math.acos(max(-1, min(1, cpsi)))
    inv = oracle.invert(r.u, r.alpha_max, psi)
    if inv is None:
        return None
    a, lf = inv[0], inv[2]
    perp = k - cpsi * rh
    nperp = np.linalg.norm(perp)
    k0 = math.cos(a) * rh + (math.sin(a) * perp / nperp if nperp > 0 else 0.0)
    eta = math.atan(r.f)
    nh = math.cos(eta) * rh - math.sin(eta) * thh          # normal tilts poleward for f > 0
    cs = float(k0 @ nh)
    if cs <= 0:
        return None
    cxi = float(k0 @ phh)
    delta = 1.0 / (r.gamma * (1 - r.beta * cxi))
    mu = delta * cs
    sq = math.sqrt(1 - r.u)
    F = sq * delta ** 3 * mu * lf * r.gamma
    z = 1.0 / (delta * sq)
    return F, z, mu


@pytest.mark.parametrize("mode", [syn.MODE_SD, syn.MODE_OS])
def test_trace_matches_vector_geometry(mode):
    spec = small_spec(mode=mode, n=8, n_fp=96)
    p = syn.params_vector(1.4, 12.5, 1.0, 0.0, 1.0, 600.0, 150.0, 0.9, 0.6, 6.1, 2.2, 0.25, 6.0, 0.38)
    for spot in (0, 1):
        for r in oracle.rings(spec, p, spot)[::3]:
            tr = oracle.trace_ring(spec, p, r)
            if not tr["visible"]:
                continue
            lo, hi = tr["inv"]
            for ifp in range(spec["n_fp"] + 1):
                if lo <= ifp <= hi:
                    continue
                v = vector_trace(spec, p, r, ifp)
                assert v is not None
                assert tr["F"][ifp] == pytest.approx(v[0], rel=1e-11, abs=1e-300)
                assert tr["z"][ifp] == pytest.approx(v[1], rel=1e-12)
                assert tr["mu"][ifp] == pytest.approx(v[2], rel=1e-11, abs=1e-15)


def test_invisible_fill_and_delay_phase():
    spec = small_spec(mode=syn.MODE_OS, n=8, n_fp=128)
    p = syn.params_vector(1.4, 12.5, 1.2, 0.0, 1.0, 600.0, 150.0, 2.0, 0.4, 6.1, 2.2, 0.25, 6.0, 0.38)
    seen_partial = False
    st = oracle.star(spec, p)
    for r in oracle.rings(spec, p, 0):
        tr = oracle.trace_ring(spec, p, r)
        if not tr["visible"]:
            continue
        lo, hi = tr["inv"]
        if lo <= hi:
            seen_partial = True
            a, b = lo - 1, hi + 1
            for ii in range(lo, hi + 1):
                t = (ii - a) / (b - a)
                assert tr["F"][ii] == 0.0 and tr["mu"][ii] == 0.0
                assert tr["z"][ii] == pytest.approx(tr["z"][a] + t * (tr["z"][b] - tr["z"][a]), rel=1e-14)
                assert tr["phio"][ii] == pytest.approx(tr["phio"][a] + t * (tr["phio"][b] - tr["phio"][a]),
                                                       rel=1e-14)
        # observed phase = emission phase + nu * delay, with the delay from
        # the (separately pinned) bending delay plus the oblate radial term
        for ifp in range(0, spec["n_fp"] + 1, 7):
            if lo <= ifp <= hi:
                continue
            phi = 2 * math.pi * ifp / spec["n_fp"]
            cpsi = math.sin(p[2]) * math.sin(r.theta) * math.cos(phi) + math.cos(p[2]) * math.cos(r.theta)
            a_ = oracle.invert(r.u, r.alpha_max, math.acos(cpsi))[0]
            cdt = r.R * oracle.tp(r.u, a_) + (st.Re - r.R + st.Rs * math.log((st.Re - st.Rs) / (r.R - st.Rs)))
            assert tr["phio"][ifp] == pytest.approx(phi / (2 * math.pi) + p[5] * cdt / syn.C_CGS, rel=1e-13)
        # observed phase is monotone over the fine grid
        assert np.all(np.diff(tr["phio"]) > 0)
    assert seen_partial
