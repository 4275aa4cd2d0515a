"""Pins of the oracle's full-surface temperature-map path (Sects. 2.6, 2.8.1).

* HEALPix geometry: 12 nside^2 patches; each ring centre lies between the
  equal-area boundaries implied by the cumulative pixel counts (a patch
  covers 4 pi / (12 nside^2) of the sphere); azimuths evenly spaced, the
  equatorial rings alternately shifted by half a pixel; north-south mirror;
* closed form: a static spherical star whose whole surface emits isotropic
  blackbody radiation at one temperature has the flux of the flux-invariance
  pin (independent of inclination and phase), approached at second order
  in the HEALPix resolution;
* symmetries: flat profile seen pole-on for a map that depends on the ring
  only; rigid rotation of the equatorial band by one pixel rolls the profile
  by P / (4 nside) phase bins; additivity over disjoint maps; at inclination
  pi / 2 a patch and its mirror image south of the equator contribute
  equally, so a map with temperature T1 in the north and T2 in the south
  equals the sum of the northern halves at T1 and at T2 (this pins the
  per-patch temperature routing).
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as syn
from test_oracle_flux import closed_form_flux


def ring_table(nside):
    return [oracle.healpix_ring(nside, i) for i in range(1, 4 * nside)]


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_healpix_geometry(nside):
    rings = ring_table(nside)
    npix = sum(n for _, n, _ in rings)
    assert npix == 12 * nside * nside
    z = np.array([r[0] for r in rings])
    assert np.all(np.diff(z) < 0)
    assert abs(z[2 * nside - 1]) < 1e-15                       # ring 2 nside is the equator
    # equal area: the boundary below ring i sits where the cap above it holds
    # exactly the pixels of rings 1..i (each pixel 1 / (12 nside^2) of 4 pi)
    cum = np.cumsum([n for _, n, _ in rings])
    zb = 1.0 - 2.0 * cum / (12.0 * nside * nside)
    zb_above = np.concatenate([[1.0], zb[:-1]])
    assert np.all(z < zb_above) and np.all(z > zb)
    assert abs(zb[-1] + 1.0) < 1e-12
    for i, (zi, n, f0) in enumerate(rings, start=1):
        assert 0.0 < f0 < 2 * math.pi / n + 1e-15               # first pixel within the first slot
        zm, nm, fm = rings[4 * nside - 1 - i]                   # mirror ring
        assert nm == n and fm == f0 and zm == -zi
        if nside <= i <= 3 * nside:
            assert n == 4 * nside
            shifted = abs(f0 - math.pi / n) < 1e-15             # centred in its slot
            assert shifted == ((i - nside) % 2 == 0)
    # in the polar caps the rings hold 4, 8, ... pixels
    assert [n for _, n, _ in rings[:nside - 1]] == [4 * k for k in range(1, nside)]


def bb_map_spec(mode, P=8, energies=(0.3, 0.8, 2.0), n_fp=128):
    e = np.array(energies, dtype=np.float64)
    return dict(mode=mode, intensity=0, n_spots=1, shape=[0, 0], n_rings=[1, 1], n_phi=[1, 1],
                shape_a=[0.0, 0.0], shape_b=[0.0, 0.0], n_fp=n_fp, n_phase=P, energy=e, t_exp=float(P),
                sigma=np.zeros(len(e)), rsp=np.eye(len(e)))


def test_whole_surface_closed_form():
    M, Re, D, lT = 1.4, 12.0, 200.0, 6.1
    ref = closed_form_flux(M, Re, D, lT, [0.3, 0.8, 2.0])
    p = syn.params_vector(M, Re, 0.7, 0.0, 0.0, 0.0, D, 0.0, 0.0, 0.0)
    errs = []
    for nside in (16, 32):
        spec = bb_map_spec(syn.MODE_SD, P=4)
        ft, _, diag = oracle.forward_map(spec, p, nside, np.full(12 * nside * nside, lT))
        err = np.max(np.abs(ft / ref - 1))
        errs.append(err)
    assert errs[1] < 2e-5, errs
    assert errs[0] / errs[1] > 3.0, errs                       # second order in nside


def test_pole_on_flat_profile():
    spec, p, _ = syn.map_config(8, n_phase=16, n_energy=16)
    p[2] = 0.0
    th, _ = syn.healpix_centres(8)
    m = np.where(th < 1.2, 6.3 - 0.5 * th, 0.0)
    ft, _, _ = oracle.forward_map(spec, p, 8, m, want_counts=False)
    assert np.max(np.abs(ft / ft[0] - 1)) < 1e-12


def test_rigid_rotation_of_equatorial_band():
    nside, P = 4, 32                                           # one pixel = P / (4 nside) = 2 bins
    spec, p, _ = syn.map_config(nside, n_phase=P, n_energy=24)
    m = syn.temperature_map(nside, "random")
    rolled = np.zeros_like(m)
    kept = np.zeros_like(m)
    off = 0
    for i, (_, n, _) in enumerate(ring_table(nside), start=1):
        seg = m[off:off + n]
        if nside <= i <= 3 * nside:
            kept[off:off + n] = seg
            rolled[off:off + n] = np.roll(seg, 1)
        off += n
    assert np.count_nonzero(kept) > 20
    ft0, _, _ = oracle.forward_map(spec, p, nside, kept, want_counts=False)
    ft1, _, _ = oracle.forward_map(spec, p, nside, rolled, want_counts=False)
    s = P // (4 * nside)
    assert np.max(np.abs(ft1 - np.roll(ft0, -s, axis=0))) <= 1e-11 * np.max(ft0)


def test_additivity_over_disjoint_maps():
    nside = 8
    spec, p, m = syn.map_config(nside, "hotspots", n_phase=16, n_energy=24)
    rng = np.random.default_rng(3)
    a = np.where(rng.uniform(size=m.size) < 0.5, m, 0.0)
    b = np.where(a > 0, 0.0, m)
    ft, _, _ = oracle.forward_map(spec, p, nside, m, want_counts=False)
    fa, _, _ = oracle.forward_map(spec, p, nside, a, want_counts=False)
    fb, _, _ = oracle.forward_map(spec, p, nside, b, want_counts=False)
    assert np.max(np.abs(fa + fb - ft)) <= 1e-12 * np.max(ft)
    # an empty map emits nothing
    f0, _, d0 = oracle.forward_map(spec, p, nside, np.zeros_like(m), want_counts=False)
    assert np.all(f0 == 0.0) and d0["n_visible_pairs"] == 0


def test_north_south_temperature_routing():
    """Inclination pi/2, rotating oblate star, atmosphere table: a patch and
    its mirror image across the equator contribute equally."""
    nside = 8
    spec, p, _ = syn.map_config(nside, n_phase=16, n_energy=24)
    p[2] = math.pi / 2
    th, ph = syn.healpix_centres(nside)
    north = th < math.pi / 2 - 1e-9
    south = th > math.pi / 2 + 1e-9
    t1 = 6.25 - 0.2 * np.cos(ph) ** 2                          # azimuth-dependent, mirrored below
    t2 = 5.9 + 0.1 * np.sin(2 * ph)
    both = np.where(north, t1, np.where(south, t2, 0.0))
    n1 = np.where(north, t1, 0.0)
    n2 = np.where(north, t2, 0.0)
    fb, _, _ = oracle.forward_map(spec, p, nside, both, want_counts=False)
    f1, _, _ = oracle.forward_map(spec, p, nside, n1, want_counts=False)
    f2, _, _ = oracle.forward_map(spec, p, nside, n2, want_counts=False)
    assert np.max(np.abs(f1 + f2 - fb)) <= 1e-12 * np.max(fb)
    # and the two halves differ, so the check has teeth
    assert np.max(np.abs(f1 - f2)) > 1e-2 * np.max(fb)
