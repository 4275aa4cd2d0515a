"""Seeded synthetic inputs shared by the FP64 CPU oracle and the HIP path.

This module holds input generators only: grids, the synthetic atmosphere
table, the interstellar cross-section, the instrument response, the
parameter vectors of each workload and the seeded parameter draws.  It holds
none of the forward model's arithmetic (ray tracing, Doppler factors,
interpolation, accumulation, folding, likelihood); both implementations
consume what is generated here and nothing else is shared between them.

The paper's own inputs are not available: the NSX-H atmosphere table, the
``tbnew`` absorption table and the NICER ARF/RMF files (Sects. 2.5, 2.7,
2.8.4).  Stand-ins with the same shapes and axis ranges are generated here:

* atmosphere: 35 logT x 11 log g x 67 mu x 166 log(E/kT) nodes over the
  ranges of Sect. 2.5, values log10(I/T^3) of a blackbody times a seeded
  limb-darkening cubic in mu whose coefficients vary linearly in logT and
  log g;
* absorption: sigma(E) = 2.4e-22 (E/keV)^-2.6 cm^2, transmission
  exp(-N_H sigma) as in Eq. (22);
* response: 300 Gaussian channels with a smooth effective-area curve,
  integrated over the model energy grid with trapezoid weights (Eqs. 23, 55).

Parameter record (16 float64 per instance):

====  ===========================================  =========
slot  meaning                                      unit
====  ===========================================  =========
0     M, gravitational mass                        M_sun
1     R_e, equatorial radius                       km
2     i, observer inclination                      rad
3     Phi, phase shift of spot 1                   cycles
4     N_H, hydrogen column                         1e20 cm^-2
5     nu, spin frequency                           Hz
6     D, distance                                  pc
7     (unused)
8     theta_1, colatitude of spot 1 centre         rad
9     zeta_1, angular radius of spot 1             rad
10    logT_1, log10 effective temperature (K)
11    (unused)
12    theta_2, colatitude of spot 2 centre         rad
13    zeta_2, (outer) angular radius of spot 2     rad
14    logT_2
15    dphi_2, longitude of spot 2 after spot 1     cycles
====  ===========================================  =========

The twelve differentiable parameters, in gradient order, are slots
0, 1, 2, 3, 4, 8, 9, 10, 12, 13, 14, 15 (``GRAD_SLOTS``).
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

# Physical constants (CGS + keV), identical on both implementations.
C_CGS = 2.99792458e10            # cm s^-1
GM_SUN = 1.3271244e26            # cm^3 s^-2
K_B_KEV = 8.617333262e-8         # keV K^-1
H_KEVS = 4.135667696e-18         # keV s
PC_CM = 3.0856775814913673e18    # cm

N_PARAM = 16
GRAD_SLOTS = (0, 1, 2, 3, 4, 8, 9, 10, 12, 13, 14, 15)
GRAD_NAMES = ("M", "R_e", "incl", "Phi", "N_H", "theta1", "zeta1", "logT1",
              "theta2", "zeta2", "logT2", "dphi2")

MODE_SD, MODE_OS = 0, 1
INTENSITY_BLACKBODY, INTENSITY_TABLE = 0, 1
SHAPE_CAP, SHAPE_ANNULUS, SHAPE_CRESCENT = 0, 1, 2

# seeds of each synthetic input
SEED_ATMOS, SEED_RESPONSE, SEED_DATA, SEED_BATCH, SEED_RES, SEED_GRAD = 11, 12, 13, 14, 15, 16
SEED_MAP = 17


def logspace(xmin: float, xmax: float, n: int) -> np.ndarray:
    """Logarithmically spaced grid, Eqs. (48)-(49)."""
    i = np.arange(n, dtype=np.float64)
    return np.exp(math.log(xmin) + (math.log(xmax) - math.log(xmin)) * i / (n - 1))


def linspace(xmin: float, xmax: float, n: int) -> np.ndarray:
    """Linearly spaced grid, Eqs. (30)-(31)."""
    i = np.arange(n, dtype=np.float64)
    return xmin + (xmax - xmin) * i / (n - 1)


# ---------------------------------------------------------------- atmosphere
def atmosphere_axes(n_t=35, n_g=11, n_mu=67, n_x=166):
    """Axes of the synthetic atmosphere table over the ranges of Sect. 2.5.

    mu nodes cluster at both ends (the paper's table has extra nodes near
    mu = 0 and mu = 1): mu_k = (1 - cos(pi k / (n_mu - 1))) / 2 with the
    first node lifted to 1e-6, the lower end of the paper's mu range.
    """
    ax_t = linspace(5.1, 6.8, n_t)
    ax_g = linspace(13.7, 14.7, n_g)
    k = np.arange(n_mu, dtype=np.float64)
    ax_mu = 0.5 * (1.0 - np.cos(np.pi * k / (n_mu - 1)))
    ax_mu[0] = 1e-6
    ax_mu[-1] = 1.0
    ax_x = linspace(-1.3, 2.0, n_x)
    return ax_t, ax_g, ax_mu, ax_x


def limb_polynomial_coeffs(seed: int = SEED_ATMOS):
    """Seeded coefficients of P(mu) = 1 + a1 mu + a2 mu^2 + a3 mu^3 with
    a_k = a_k0 + a_kT (logT - 6) + a_kg (log g - 14.2).  Draws whose P drops
    to 0.05 or below anywhere on mu in [0, 1] over the table's logT, log g
    ranges are rejected."""
    rng = np.random.default_rng(seed)
    mus = np.linspace(0.0, 1.0, 201)
    ax_t, ax_g, _, _ = atmosphere_axes()
    while True:
        a0 = np.array([rng.uniform(0.5, 2.0), rng.uniform(-0.5, 0.5), rng.uniform(-0.2, 0.2)])
        aT = rng.uniform(-0.1, 0.1, 3)
        ag = rng.uniform(-0.1, 0.1, 3)
        ok = True
        for lt in (ax_t[0], ax_t[-1]):
            for lg in (ax_g[0], ax_g[-1]):
                a = a0 + aT * (lt - 6.0) + ag * (lg - 14.2)
                p = 1.0 + a[0] * mus + a[1] * mus ** 2 + a[2] * mus ** 3
                if p.min() <= 0.05:
                    ok = False
        if ok:
            return a0, aT, ag


def atmosphere_table(seed: int = SEED_ATMOS, n_t=35, n_g=11, n_mu=67, n_x=166):
    """Synthetic stand-in for the NSX-H table: log10(I T^-3) on the 4D grid.

    V = (2 k_B^3 / (h^3 c^2)) y^3 / (e^y - 1) * P(mu; logT, log g), y = 10^x,
    so that T^3 V is the blackbody photon-energy intensity of App. C,
    Eq. (C.5), times the limb-darkening factor P.  Returned as float64
    array [n_t, n_g, n_mu, n_x] of log10 V plus the four axes.
    """
    ax_t, ax_g, ax_mu, ax_x = atmosphere_axes(n_t, n_g, n_mu, n_x)
    a0, aT, ag = limb_polynomial_coeffs(seed)
    y = 10.0 ** ax_x
    # y^3/(e^y-1) computed as y^3 e^-y / (1 - e^-y) to stay finite at y = 100
    bb = y ** 3 * np.exp(-y) / (-np.expm1(-y))
    pref = 2.0 * K_B_KEV ** 3 / (H_KEVS ** 3 * C_CGS ** 2)
    lt = ax_t[:, None, None]
    lg = ax_g[None, :, None]
    mu = ax_mu[None, None, :]
    a1 = a0[0] + aT[0] * (lt - 6.0) + ag[0] * (lg - 14.2)
    a2 = a0[1] + aT[1] * (lt - 6.0) + ag[1] * (lg - 14.2)
    a3 = a0[2] + aT[2] * (lt - 6.0) + ag[2] * (lg - 14.2)
    p = 1.0 + a1 * mu + a2 * mu ** 2 + a3 * mu ** 3            # [t, g, mu]
    v = pref * p[..., None] * bb[None, None, None, :]
    return np.log10(v), (ax_t, ax_g, ax_mu, ax_x)


def atmosphere_table_multilinear(n_t=35, n_g=11, n_mu=67, n_x=166):
    """Synthetic table that is a product of linear functions of its four
    axes, V = c (1 + 0.3 (logT - 6)) (1 + 0.2 (log g - 14.2)) (1 + 0.8 mu)
    (2.5 - x), positive over the axes' ranges.  Every interpolation
    strategy of Sect. 4 reproduces it exactly, so a model built on it has no
    kinks from interpolation stencils: what is left of the forward model's
    piecewise structure is the fine-phase interpolation (Eq. 46) and
    visibility.  Used for gradient checks at tight tolerance.  Same axes
    and layout as atmosphere_table (log10 V)."""
    ax_t, ax_g, ax_mu, ax_x = atmosphere_axes(n_t, n_g, n_mu, n_x)
    pref = 0.03 * 2.0 * K_B_KEV ** 3 / (H_KEVS ** 3 * C_CGS ** 2)
    v = (pref * (1.0 + 0.3 * (ax_t[:, None, None, None] - 6.0)) * (1.0 + 0.2 * (ax_g[None, :, None, None] - 14.2))
         * (1.0 + 0.8 * ax_mu[None, None, :, None]) * (2.5 - ax_x[None, None, None, :]))
    return np.log10(v), (ax_t, ax_g, ax_mu, ax_x)


def atmosphere_table_steep_limb(n_t=35, n_g=11, n_mu=67, n_x=166):
    """Synthetic table with a limb far steeper than the mu grid resolves,
    for the interpolation-overshoot diagnostics of Sect. 4: the blackbody
    factor of atmosphere_table times L(mu) = 1e-6 + tanh(mu / 0.004)^4
    (rising from ~0 to ~1 across the first five mu nodes) times a mild
    linear logT / log g trend.  Same axes and layout as atmosphere_table."""
    ax_t, ax_g, ax_mu, ax_x = atmosphere_axes(n_t, n_g, n_mu, n_x)
    y = 10.0 ** ax_x
    bb = y ** 3 * np.exp(-y) / (-np.expm1(-y))
    pref = 2.0 * K_B_KEV ** 3 / (H_KEVS ** 3 * C_CGS ** 2)
    trend = 1.0 + 0.1 * (ax_t[:, None, None] - 6.0) + 0.05 * (ax_g[None, :, None] - 14.2)
    limb = 1e-6 + np.tanh(ax_mu / 0.004) ** 4
    v = pref * (trend * limb[None, None, :])[..., None] * bb[None, None, None, :]
    return np.log10(v), (ax_t, ax_g, ax_mu, ax_x)


def interp_test_geometry(test: int, n_cells=16, n_phase=64, n_energy=32):
    """The single small hotspot of the interpolation tests of Sect. 4
    (Table 3): M = 1.4, R_e = 12 km, 600 Hz, T = 1e6 K, D = 150 pc, spot
    radius 0.01 rad; test 1: colatitude 1.983 rad seen from i = 0.01 rad,
    test 2: colatitude pi - 0.01 rad seen from i = 0.964 rad.  Oblate star,
    steep-limb synthetic table, no absorption."""
    th, inc = (1.983, 0.01) if test == 1 else (math.pi - 0.01, 0.964)
    spec = _base_spec(n_spots=1, shape=[SHAPE_CAP, SHAPE_CAP], n_rings=[n_cells, n_cells],
                      n_phi=[n_cells, n_cells], shape_a=[0.0, 0.0], n_phase=n_phase,
                      energy=logspace(0.2, 3.0, n_energy), precision="f32")
    logi, axes = atmosphere_table_steep_limb()
    spec["atmos_logI"] = logi
    spec["atmos_axes"] = axes
    spec["sigma"] = np.zeros(n_energy)
    spec["rsp"] = gaussian_response(spec["energy"])
    params = params_vector(1.4, 12.0, inc, 0.0, 0.0, 600.0, 150.0, th, 0.01, 6.0)
    return spec, params


# ------------------------------------------------------- absorption, response
def sigma_ism(energy_kev: np.ndarray) -> np.ndarray:
    """Stand-in photo-absorption cross-section per H atom [cm^2]."""
    return 2.4e-22 * np.asarray(energy_kev, dtype=np.float64) ** (-2.6)


def gaussian_response(energy_kev: np.ndarray, n_chan: int = 300, seed: int = SEED_RESPONSE):
    """Stand-in for ARF x RMF folded onto the model grid, RSP[e, c] in cm^2 keV.

    Channel c collects [0.15 + 0.01 c, 0.15 + 0.01 (c + 1)] keV.  A photon of
    energy E lands at a Gaussian-distributed pulse height of width
    s0 sqrt(E/keV); the effective area is A0 exp(-((ln E - ln 1.5)/0.8)^2).
    The model-energy integral of Eq. (23) uses trapezoid weights on the
    (log-spaced) energy grid.
    """
    rng = np.random.default_rng(seed)
    s0 = rng.uniform(0.03, 0.06)
    a0 = rng.uniform(900.0, 1100.0)
    e = np.asarray(energy_kev, dtype=np.float64)
    de = np.empty_like(e)
    de[1:-1] = 0.5 * (e[2:] - e[:-2])
    de[0] = 0.5 * (e[1] - e[0])
    de[-1] = 0.5 * (e[-1] - e[-2])
    area = a0 * np.exp(-((np.log(e) - math.log(1.5)) / 0.8) ** 2)
    cc = 0.15 + 0.01 * (np.arange(n_chan) + 0.5)
    sig = s0 * np.sqrt(e)
    g = np.exp(-0.5 * ((cc[None, :] - e[:, None]) / sig[:, None]) ** 2) / (sig[:, None] * math.sqrt(2 * math.pi))
    return (area * de)[:, None] * g * 0.01


# ------------------------------------------------------------------ workloads
def params_vector(M, Re, incl, Phi, NH, nu, D, th1, z1, lT1, th2=0.0, z2=0.0, lT2=0.0, dphi2=0.0):
    p = np.zeros(N_PARAM, dtype=np.float64)
    p[0], p[1], p[2], p[3], p[4], p[5], p[6] = M, Re, incl, Phi, NH, nu, D
    p[8], p[9], p[10] = th1, z1, lT1
    p[12], p[13], p[14], p[15] = th2, z2, lT2, dphi2
    return p


def _base_spec(**kw):
    spec = dict(mode=MODE_OS, intensity=INTENSITY_TABLE, n_spots=2,
                shape=[SHAPE_CAP, SHAPE_ANNULUS], n_rings=[128, 128], n_phi=[128, 128],
                shape_a=[0.0, 0.4], shape_b=[0.0, 0.0], n_fp=192, n_phase=128,
                energy=logspace(0.2, 3.0, 256), t_exp=1.0e6, n_alpha=512)
    spec.update(kw)
    return spec


def attach_atmosphere(spec, seed: int = SEED_ATMOS):
    logi, axes = atmosphere_table(seed)
    spec["atmos_logI"] = logi
    spec["atmos_axes"] = axes
    return spec


def attach_instrument(spec, n_chan=300, seed: int = SEED_RESPONSE):
    spec["sigma"] = sigma_ism(spec["energy"])
    spec["rsp"] = gaussian_response(spec["energy"], n_chan, seed)
    return spec


def config0():
    """Plain forward model in FP64: spherical star (Schwarzschild + Doppler),
    one circular spot, isotropic blackbody, identity response, no absorption."""
    n_e = 32
    spec = _base_spec(mode=MODE_SD, intensity=INTENSITY_BLACKBODY, n_spots=1,
                      shape=[SHAPE_CAP, SHAPE_CAP], n_rings=[32, 32], n_phi=[32, 32],
                      shape_a=[0.0, 0.0], n_fp=192, n_phase=32,
                      energy=logspace(0.2, 3.0, n_e), t_exp=32.0, precision="f64")
    spec["sigma"] = np.zeros(n_e)
    spec["rsp"] = np.eye(n_e)
    params = params_vector(1.4, 12.0, math.radians(60.0), 0.0, 0.0, 200.0, 200.0,
                           math.radians(45.0), 0.2, 6.1)
    return spec, params


def config1(n_cells=128, n_phase=128, n_energy=256):
    """Plain high-fidelity model: oblate star at 600 Hz, a circular cap and a
    non-antipodal annulus, synthetic atmosphere, absorption and response."""
    spec = _base_spec(n_rings=[n_cells, n_cells], n_phi=[n_cells, n_cells],
                      n_phase=n_phase, energy=logspace(0.2, 3.0, n_energy), precision="f32")
    attach_atmosphere(spec)
    attach_instrument(spec)
    params = params_vector(1.4, 12.5, math.radians(60.0), 0.05, 1.0, 600.0, 150.0,
                           math.pi / 4, 0.2, 6.1, 2.2, 0.25, 6.0, 0.38)
    return spec, params


def config2(n_cells=512, n_phase=256, n_fp=512):
    """Extreme geometry at compactness GM/(R c^2) = 0.28: a cap of angular
    radius 1.2 rad straddling the pole and a small crescent near grazing."""
    re_km = 12.5
    m_sun = 0.28 * re_km * 1e5 * C_CGS ** 2 / GM_SUN
    spec = _base_spec(shape=[SHAPE_CAP, SHAPE_CRESCENT], n_rings=[n_cells, n_cells],
                      n_phi=[n_cells, n_cells], shape_a=[0.0, 0.8], shape_b=[0.0, 0.4],
                      n_fp=n_fp, n_phase=n_phase, energy=logspace(0.2, 3.0, 256), precision="f32")
    attach_atmosphere(spec)
    attach_instrument(spec)
    params = params_vector(m_sun, re_km, math.radians(85.0), 0.0, 1.0, 600.0, 150.0,
                           0.3, 1.2, 6.0, math.radians(170.0), 0.05, 6.2, 0.3)
    return spec, params


def compactness(params) -> np.ndarray:
    p = np.atleast_2d(params)
    return p[:, 0] * GM_SUN / (C_CGS ** 2 * p[:, 1] * 1e5)


def spots_overlap(p) -> bool:
    """True when the two spot caps overlap (centre separation < zeta1+zeta2)."""
    c = (math.cos(p[8]) * math.cos(p[12]) + math.sin(p[8]) * math.sin(p[12])
         * math.cos(2 * math.pi * p[15]))
    sep = math.acos(max(-1.0, min(1.0, c)))
    return sep < p[9] + p[13]


def config3_draws(n=1024, seed=SEED_BATCH, res_seed=SEED_RES):
    """Seeded sampler-like parameter vectors and per-instance spot resolutions
    (cells per side, from {64, 128, 256, 512}); draws above compactness 0.28
    or with overlapping spots are rejected and redrawn."""
    rng = np.random.default_rng(seed)
    out = np.zeros((n, N_PARAM))
    k = 0
    while k < n:
        p = params_vector(rng.uniform(1.0, 2.2), rng.uniform(9.0, 15.0),
                          rng.uniform(0.05, math.pi - 0.05), rng.uniform(0.0, 1.0), 1.0, 600.0, 150.0,
                          rng.uniform(0.05, math.pi - 0.05), rng.uniform(0.01, 1.0),
                          rng.uniform(5.8, 6.6),
                          rng.uniform(0.05, math.pi - 0.05), rng.uniform(0.01, 1.0),
                          rng.uniform(5.8, 6.6), rng.uniform(0.0, 1.0))
        if compactness(p)[0] > 0.28 or spots_overlap(p):
            continue
        out[k] = p
        k += 1
    res = np.random.default_rng(res_seed).choice(np.array([64, 128, 256, 512]), size=n)
    return out, res


def config4_draws(n=256, seed=SEED_GRAD):
    """Parameter vectors within +-5% of the config-1 truth over the twelve
    differentiable slots (overlap and compactness rejections as above)."""
    _, truth = config1()
    rng = np.random.default_rng(seed)
    out = np.zeros((n, N_PARAM))
    k = 0
    while k < n:
        p = truth.copy()
        for s in GRAD_SLOTS:
            p[s] = truth[s] * (1.0 + rng.uniform(-0.05, 0.05))
        if compactness(p)[0] > 0.28 or spots_overlap(p):
            continue
        out[k] = p
        k += 1
    return out


# ---------------------------------------------------------------------------
# Full-surface temperature maps on HEALPix (Sects. 2.6, 2.8.1).  The paper's
# physics-motivated generator (return-current heating of an off-centred
# dipole) is not available; smooth synthetic maps with a hot polar-cap-like
# region with a radial temperature gradient and a cooler arc stand in for it.
# The patch centres below place those features only; the oracle and the HIP
# path each compute the HEALPix geometry themselves.
# ---------------------------------------------------------------------------
def healpix_centres(nside: int):
    """(colatitude, azimuth) of every HEALPix patch centre, ring order: rings
    from the north pole, pixels by increasing azimuth."""
    th, ph = [], []
    for i in range(1, 4 * nside):
        m = min(i, 4 * nside - i)
        if m < nside:
            z = 1.0 - m * m / (3.0 * nside * nside)
            n = 4 * m
            phi = math.pi / (2.0 * m) * (np.arange(n) + 0.5)
        else:
            z = 4.0 / 3.0 - 2.0 * m / (3.0 * nside)
            n = 4 * nside
            phi = math.pi / (2.0 * nside) * (np.arange(n) + 1.0 - ((m - nside + 1) % 2) / 2.0)
        if i > 2 * nside:
            z = -z
        th.append(np.full(n, math.acos(z)))
        ph.append(phi)
    return np.concatenate(th), np.concatenate(ph)


def _angular_distance(th, ph, th0, ph0):
    c = np.cos(th) * math.cos(th0) + np.sin(th) * math.sin(th0) * np.cos(ph - ph0)
    return np.arccos(np.clip(c, -1.0, 1.0))


def temperature_map(nside: int, kind: str = "hotspots", seed: int = SEED_MAP) -> np.ndarray:
    """log10 T [K] per HEALPix patch (ring order); 0 marks an inactive patch.

    hotspots  a polar-cap-like region (centre colatitude 0.5 rad, azimuth 0,
              radius 0.45 rad, logT falling from 6.35 at the centre to 5.95
              at the rim) and an arc (annulus 0.12-0.30 rad around colatitude
              2.45 rad, azimuth 2.5 rad, logT 5.95-6.10); the rest inactive;
    full      every patch active: a smooth background around logT 5.6 with
              the hotspots on top (the larger of the two);
    random    seeded: 30% of the patches active with logT uniform in
              [4.8, 7.0], beyond the table's range on both sides.
    """
    th, ph = healpix_centres(nside)
    if kind == "random":
        rng = np.random.default_rng(seed)
        lt = rng.uniform(4.8, 7.0, th.size)
        return np.where(rng.uniform(size=th.size) < 0.3, lt, 0.0)
    d1 = _angular_distance(th, ph, 0.5, 0.0)
    d2 = _angular_distance(th, ph, 2.45, 2.5)
    hot = np.zeros(th.size)
    cap = d1 <= 0.45
    hot[cap] = 6.35 - 0.40 * (d1[cap] / 0.45) ** 2
    arc = (d2 >= 0.12) & (d2 <= 0.30)
    hot[arc] = 5.95 + 0.15 * np.sin(math.pi * (d2[arc] - 0.12) / 0.18)
    if kind == "hotspots":
        return hot
    if kind == "full":
        bg = 5.55 + 0.10 * np.cos(th) ** 2 + 0.05 * np.sin(th) * np.cos(ph - 1.0)
        return np.maximum(bg, hot)
    raise ValueError(kind)


def map_config(nside: int = 64, kind: str = "full", n_phase: int = 128, n_energy: int = 256):
    """Full-surface temperature map workload: the config-1 star (oblate,
    600 Hz, M = 1.4, R_e = 12.5 km, i = 60 deg, 150 pc), the synthetic
    atmosphere, absorption and response, and a HEALPix map of nside."""
    spec = _base_spec(n_phase=n_phase, energy=logspace(0.2, 3.0, n_energy), precision="f32", n_side=nside)
    attach_atmosphere(spec)
    attach_instrument(spec)
    params = params_vector(1.4, 12.5, math.radians(60.0), 0.05, 1.0, 600.0, 150.0, 0.0, 0.0, 0.0)
    return spec, params, temperature_map(nside, kind)


def poisson_data(counts: np.ndarray, seed: int = SEED_DATA) -> np.ndarray:
    """Seeded Poisson draw of observed counts from expected counts."""
    rng = np.random.default_rng(seed)
    return rng.poisson(np.asarray(counts, dtype=np.float64)).astype(np.int32)


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]
