"""End-to-end pins of the oracle's forward model (Sects. 2.5, 2.8.3, App. C).

* flux invariance: a static spherical star whose whole visible hemisphere
  emits isotropic blackbody radiation has the closed-form flux
  F(E) = pi R^2 / (D^2 (1-u)) * 2 E^2 / (h^3 c^2) / (exp(E / (k T sqrt(1-u))) - 1)
  (integral of cos(alpha) d cos(alpha) over the visible disc is 1/2), with
  second-order convergence in the number of rings;
* symmetries: flat profile at zero inclination, mirror symmetry of a static
  star about the spot meridian, antipodal symmetry (spot at (pi - theta,
  phi + pi) seen from pi - i is the original shifted by half a cycle),
  exact phase-roll equivariance, additivity of spots;
* brute force: for a handful of cells, the continuum flux obtained by
  root-finding the emission azimuth of each observed phase and evaluating
  the ray with radial quadratures and 3D vectors (no tables, no fine-phase
  resampling) matches the oracle's shift-and-add at high N_fp.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
import synthetic as syn


def spec_bb(mode, n_rings, n_phi, n_fp=192, P=16, energies=(0.3, 0.8, 2.0), n_spots=1, shape=(0, 0)):
    e = np.array(energies, dtype=np.float64)
    return dict(mode=mode, intensity=0, n_spots=n_spots, shape=list(shape), n_rings=[n_rings, n_rings],
                n_phi=[n_phi, n_phi], shape_a=[0.0, 0.4], shape_b=[0.0, 0.0], n_fp=n_fp, n_phase=P,
                energy=e, t_exp=float(P), sigma=np.zeros(len(e)), rsp=np.eye(len(e)))


def closed_form_flux(M, Re_km, D_pc, logT, E):
    GM = M * syn.GM_SUN
    R = Re_km * 1e5
    u = 2 * GM / (syn.C_CGS ** 2 * R)
    D = D_pc * syn.PC_CM
    T = 10 ** logT
    E = np.asarray(E)
    return (math.pi * R * R / (D * D * (1 - u)) * 2 * E ** 2 / (syn.H_KEVS ** 3 * syn.C_CGS ** 2)
            / np.expm1(E / (syn.K_B_KEV * T * math.sqrt(1 - u))))


def test_flux_invariance_static_sphere():
    M, Re, D, lT = 1.4, 12.0, 200.0, 6.1
    u = 2 * M * syn.GM_SUN / (syn.C_CGS ** 2 * Re * 1e5)
    psimax = oracle.psi(u, math.pi / 2)
    ref = closed_form_flux(M, Re, D, lT, [0.3, 0.8, 2.0])
    errs = []
    for n in (32, 64):
        spec = spec_bb(syn.MODE_SD, n, 4, n_fp=64, P=4)
        p = syn.params_vector(M, Re, 0.0, 0.0, 0.0, 0.0, D, 0.0, psimax, lT)
        ft, _, _ = oracle.forward(spec, p)
        # phase independent to rounding
        assert np.max(np.abs(ft - ft[0])) <= 1e-13 * np.max(ft)
        errs.append(np.max(np.abs(ft[0] / ref - 1)))
    assert errs[1] < 2e-4
    assert 3.0 < errs[0] / errs[1] < 5.0          # second-order convergence


@pytest.mark.parametrize("mode", [syn.MODE_SD, syn.MODE_OS])
def test_flat_profile_at_zero_inclination(mode):
    spec = spec_bb(mode, 8, 8)
    p = syn.params_vector(1.4, 12.0, 0.0, 0.17, 0.0, 400.0, 200.0, 0.7, 0.3, 6.1)
    ft, _, _ = oracle.forward(spec, p)
    assert np.max(np.abs(ft / ft[0] - 1)) < 1e-12


@pytest.mark.parametrize("mode", [syn.MODE_SD, syn.MODE_OS])
def test_static_mirror_symmetry(mode):
    spec = spec_bb(mode, 8, 8, P=16)
    p = syn.params_vector(1.4, 12.0, 1.1, 0.0, 0.0, 0.0, 200.0, 1.3, 0.4, 6.1)
    ft, _, _ = oracle.forward(spec, p)
    assert np.max(np.abs(ft - ft[::-1])) <= 1e-12 * np.max(ft)


@pytest.mark.parametrize("mode", [syn.MODE_SD, syn.MODE_OS])
def test_antipodal_symmetry(mode):
    spec = spec_bb(mode, 8, 8, P=16)
    p = syn.params_vector(1.4, 12.0, 1.1, 0.1, 0.0, 300.0, 200.0, 0.9, 0.3, 6.1)
    # reflection through the equatorial plane: spot at pi - theta seen from
    # pi - i gives the identical profile
    q = p.copy()
    q[2] = math.pi - p[2]
    q[8] = math.pi - p[8]
    a, _, _ = oracle.forward(spec, p)
    b, _, _ = oracle.forward(spec, q)
    np.testing.assert_allclose(b, a, rtol=1e-11, atol=1e-12 * a.max())
    # antipodal spot (pi - theta, phi + pi) seen from i = original seen from
    # pi - i shifted by half a cycle
    r = p.copy()
    r[8] = math.pi - p[8]
    r[3] = p[3] + 0.5
    c, _, _ = oracle.forward(spec, r)
    q2 = p.copy()
    q2[2] = math.pi - p[2]
    d, _, _ = oracle.forward(spec, q2)
    np.testing.assert_allclose(c, np.roll(d, 8, axis=0), rtol=1e-11, atol=1e-12 * d.max())
    # two identical antipodal spots seen at i = pi/2: period one half
    spec2 = spec_bb(mode, 8, 8, P=16, n_spots=2)
    r = syn.params_vector(1.4, 12.0, math.pi / 2, 0.1, 0.0, 300.0, 200.0, 0.9, 0.3, 6.1,
                          math.pi - 0.9, 0.3, 6.1, 0.5)
    c, _, _ = oracle.forward(spec2, r)
    np.testing.assert_allclose(c, np.roll(c, 8, axis=0), rtol=1e-11)


def test_phase_roll_and_additivity():
    spec = spec_bb(syn.MODE_OS, 8, 8, P=16, n_spots=2, shape=(0, 1))
    p = syn.params_vector(1.4, 12.0, 1.1, 0.1, 0.0, 300.0, 200.0, 0.9, 0.3, 6.1, 2.0, 0.4, 6.0, 0.3)
    a, _, _ = oracle.forward(spec, p)
    q = p.copy()
    q[3] += 3.0 / 16
    b, _, _ = oracle.forward(spec, q)
    np.testing.assert_allclose(b, np.roll(a, 3, axis=0), rtol=1e-11, atol=1e-13 * a.max())
    # two spots = spot one + spot two
    s1 = dict(spec, n_spots=1)
    f1, _, _ = oracle.forward(s1, p)
    s2 = dict(spec, n_spots=1, shape=[1, 1], shape_a=[0.4, 0.4])
    p2 = p.copy()
    p2[8:12] = p[12:16]
    p2[3] = p[3] + p[15]          # spot 2 longitude in its own frame
    f2, _, _ = oracle.forward(s2, p2)
    np.testing.assert_allclose(a, f1 + f2, rtol=1e-12, atol=1e-14 * a.max())


# ----------------------------------------------------------------- brute force
def _psi_w(u, a):
    p2 = (u * math.sqrt(1 - u) / math.sin(a)) ** 2
    return integrate.quad(lambda w: 1 / math.sqrt(p2 - w * w + w ** 3), 0, u, epsabs=0, epsrel=1e-13, limit=200)[0]


def _alpha_of_psi(u, psi):
    return optimize.brentq(lambda a: _psi_w(u, a) - psi, 1e-14, math.pi / 2 - 1e-9, xtol=1e-15, rtol=1e-15)


def _tp_w(u, a):
    bb = (math.sin(a) / (u * math.sqrt(1 - u))) ** 2
    f = lambda w: u / (w * w * (1 - w)) * (1 / math.sqrt(1 - bb * w * w * (1 - w)) - 1)
    return integrate.quad(f, 0, u, epsabs=0, epsrel=1e-13, limit=200)[0]


class Continuum:
    """Direct evaluation of one surface element at a given emission azimuth."""

    def __init__(self, p, mode, theta, Rs, Re, o2, nu):
        self.p, self.mode, self.th = p, mode, theta
        self.R = Re * (1 + o2 * math.cos(theta) ** 2)
        Rt = -2 * Re * o2 * math.cos(theta) * math.sin(theta)
        self.u = Rs / self.R
        self.f = Rt / (self.R * math.sqrt(1 - self.u))
        self.beta = 2 * math.pi * nu * self.R * math.sin(theta) / (syn.C_CGS * math.sqrt(1 - self.u))
        self.gamma = 1 / math.sqrt(1 - self.beta ** 2)
        self.cdt_obl = Re - self.R + Rs * math.log((Re - Rs) / (self.R - Rs))
        self.nu = nu

    def ray(self, phi):
        i = self.p[2]
        th = self.th
        k = np.array([math.sin(i), 0.0, math.cos(i)])
        rh = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
        thh = np.array([math.cos(th) * math.cos(phi), math.cos(th) * math.sin(phi), -math.sin(th)])
        phh = np.array([-math.sin(phi), math.cos(phi), 0.0])
        cpsi = float(k @ rh)
        psi = math.acos(cpsi)
        a = _alpha_of_psi(self.u, psi)
        h = 1e-6
        ap = _alpha_of_psi(self.u, math.acos(cpsi + h))
        am = _alpha_of_psi(self.u, math.acos(cpsi - h))
        lf = (math.cos(ap) - math.cos(am)) / (2 * h)
        perp = k - cpsi * rh
        k0 = math.cos(a) * rh + math.sin(a) * perp / np.linalg.norm(perp)
        eta = math.atan(self.f)
        nh = math.cos(eta) * rh - math.sin(eta) * thh
        cs = float(k0 @ nh)
        cxi = float(k0 @ phh)
        delta = 1 / (self.gamma * (1 - self.beta * cxi))
        sq = math.sqrt(1 - self.u)
        F = sq * delta ** 3 * delta * cs * lf * self.gamma
        z = 1 / (delta * sq)
        cdt = self.R * _tp_w(self.u, a) + self.cdt_obl
        return F, z, cdt / syn.C_CGS

    def observed(self, phi_c, Phi):
        """Emission azimuth phi of the photon observed at phase Phi:
        (phi - phi_c)/2pi + nu dt(phi) = Phi (mod 1)."""
        g = lambda ph: (ph - phi_c) / (2 * math.pi) + self.nu * self.ray(ph)[2] - Phi
        x0 = phi_c + 2 * math.pi * Phi
        ph = optimize.brentq(g, x0 - 2 * math.pi * 0.2, x0 + 0.1, xtol=1e-14)
        return self.ray(ph)


@pytest.mark.parametrize("mode", [syn.MODE_SD, syn.MODE_OS])
def test_brute_force_continuum(mode):
    nr, nphi, P = 2, 3, 5
    energies = (0.4, 1.0, 2.5)
    spec = spec_bb(mode, nr, nphi, n_fp=4096, P=P, energies=energies)
    p = syn.params_vector(1.4, 12.0, 1.0, 0.13, 0.0, 400.0, 200.0, 0.55, 0.08, 6.1)
    ft, _, _ = oracle.forward(spec, p)
    GM = p[0] * syn.GM_SUN
    Re = p[1] * 1e5
    Rs = 2 * GM / syn.C_CGS ** 2
    x = GM / (syn.C_CGS ** 2 * Re)
    Ob = 2 * math.pi * p[5] * math.sqrt(Re ** 3 / GM)
    o2 = Ob ** 2 * (-0.788 + 1.030 * x) if mode == syn.MODE_OS else 0.0
    D = p[6] * syn.PC_CM
    T = 10 ** p[10]
    tc, z = p[8], p[9]
    ref = np.zeros_like(ft)
    for r in range(nr):
        e0, e1 = tc - z + 2 * z * r / nr, tc - z + 2 * z * (r + 1) / nr
        th = 0.5 * (e0 + e1)
        dcos = math.cos(e0) - math.cos(e1)
        arg = (math.cos(z) - math.cos(th) * math.cos(tc)) / (math.sin(th) * math.sin(tc))
        hw = math.acos(max(-1, min(1, arg)))
        dphi = 2 * hw / nphi
        el = Continuum(p, mode, th, Rs, Re, o2, p[5])
        w = el.R ** 2 * math.sqrt(1 + el.f ** 2) * dcos * dphi / D ** 2
        for j in range(nphi):
            phi_c = -2 * math.pi * p[3] + (-hw + (j + 0.5) * dphi)
            for k in range(P):
                F, zz, _ = el.observed(phi_c, (k + 0.5) / P)
                for e, E in enumerate(energies):
                    Ep = zz * E
                    I = 2 * Ep ** 3 / (syn.H_KEVS ** 3 * syn.C_CGS ** 2) / math.expm1(Ep / (syn.K_B_KEV * T))
                    ref[k, e] += w * F * I / E
    np.testing.assert_allclose(ft, ref, rtol=3e-6)
