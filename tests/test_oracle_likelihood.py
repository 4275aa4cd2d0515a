"""Pins of the oracle's absorption, response fold and Poisson likelihood
(Sects. 2.7, 2.8.4, 6), and of its finite-difference gradient.

* log-likelihood against scipy.stats.poisson.logpmf (an independent
  library routine) and its special cases d = 0 and m <= 0;
* fold with an identity response and no absorption reduces to the photon
  flux times the exposure per phase bin; a single-energy response isolates
  the transmission exp(-N_H sigma) of Eq. (22);
* the FD gradient is consistent under step halving (Richardson check).
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synthetic as syn


def test_loglike_vs_scipy():
    rng = np.random.default_rng(5)
    m = rng.uniform(0.01, 50.0, size=5000)
    d = rng.poisson(m).astype(np.int32)
    want = stats.poisson.logpmf(d, m).sum()
    assert oracle.loglike_from_counts(m, d) == pytest.approx(want, rel=1e-13)
    assert oracle.loglike_from_counts(np.array([2.5]), np.array([0], np.int32)) == pytest.approx(-2.5)
    assert oracle.loglike_from_counts(np.array([0.0]), np.array([3], np.int32)) == -math.inf
    assert oracle.loglike_from_counts(np.array([0.0]), np.array([0], np.int32)) == 0.0


def small_cfg1():
    spec, p = syn.config1(n_cells=8, n_phase=16, n_energy=32)
    return spec, p


def test_fold_identity_and_transmission():
    spec, p = small_cfg1()
    E = len(spec["energy"])
    s = dict(spec, rsp=np.eye(E), sigma=np.zeros(E), t_exp=16.0)
    ft, cnt, _ = oracle.forward(s, p)
    np.testing.assert_allclose(cnt, ft, rtol=1e-14)      # T_exp / P = 1
    # single energy column: counts = T_exp/P * Ft[:, e] * exp(-N_H sigma_e) * rsp
    e = 7
    rsp = np.zeros((E, 1))
    rsp[e, 0] = 3.0
    s2 = dict(spec, rsp=rsp, t_exp=1.6e3)
    ft2, cnt2, _ = oracle.forward(s2, p)
    att = math.exp(-p[4] * 1e20 * spec["sigma"][e])
    np.testing.assert_allclose(cnt2[:, 0], 1.6e3 / 16 * ft2[:, e] * att * 3.0, rtol=1e-14)
    assert 0.0 < att < 1.0


def test_fd_gradient_richardson():
    spec, p = small_cfg1()
    os_ = oracle.OracleSpec(spec)
    _, cnt, _ = oracle.forward(os_, p)
    data = syn.poisson_data(cnt)
    q = p.copy()
    # off the table nodes in logT (linear there, so the likelihood has a kink
    # in logT at every node; see the gradient notes)
    q[[0, 2, 9, 10]] *= (1.02, 0.98, 1.03, 1.003)
    slots = (0, 2, 3, 9, 10, 15)
    g1 = oracle.fd_gradient(os_, q, data, slots, rel_step=1e-4)
    g2 = oracle.fd_gradient(os_, q, data, slots, rel_step=5e-5)
    # piecewise-cubic Lagrange in x and mu and linear phase/logT/log g
    # interpolation make the likelihood C0 with many small slope jumps, so
    # central differences agree to O(h) ~ 1e-4 relative, 1e-6 of |g|max
    np.testing.assert_allclose(g1, g2, rtol=1e-4, atol=1e-6 * np.abs(g1).max())
    assert np.all(np.abs(g1) > 0)


def test_fd_gradient_counts_pins():
    """The chain-rule differences (counts differenced, contracted with
    d logL / d m = d / m - 1): the N_H component against its closed form
    (N_H enters only through exp(-N_H sigma), so d m / d N_H =
    -1e20 T_exp / P (F_t sigma exp(-N_H sigma)) RSP from the oracle's flux),
    and every component against the plain differences of logL where both
    converge (multilinear table, no stencil kinks)."""
    spec, p = syn.config1(n_cells=8, n_phase=16, n_energy=32)
    logi, axes = syn.atmosphere_table_multilinear()
    spec["atmos_logI"], spec["atmos_axes"] = logi, axes
    os_ = oracle.OracleSpec(spec)
    _, cnt, _ = oracle.forward(os_, p)
    data = syn.poisson_data(cnt)
    q = syn.config4_draws(1)[0]
    g = oracle.fd_gradient_counts(os_, q, data, syn.GRAD_SLOTS, rel_step=1e-6)
    ft, m, _ = oracle.forward(os_, q)
    sig = spec["sigma"]
    att = np.exp(-q[4] * 1e20 * sig)
    dm = -1e20 * (ft * sig * att) @ spec["rsp"] * (spec["t_exp"] / 16)
    gm = np.where(data > 0, data / m, 0.0) - 1.0
    assert g[4] == pytest.approx(float(np.sum(gm * dm)), rel=1e-8)
    gl = oracle.fd_gradient(os_, q, data, syn.GRAD_SLOTS, rel_step=3e-6)
    np.testing.assert_allclose(g, gl, rtol=2e-5)
    # background: the contraction uses d / (m + b) - 1
    b = np.full_like(m, 0.5 * m.mean())
    gb = oracle.fd_gradient_counts(os_, q, data, (4,), rel_step=1e-6, background=b)
    gmb = np.where(data > 0, data / (m + b), 0.0) - 1.0
    assert gb[0] == pytest.approx(float(np.sum(gmb * dm)), rel=1e-8)
