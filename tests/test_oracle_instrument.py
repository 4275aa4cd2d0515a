"""Pins of the oracle's instrument pipeline (Sect. 2.8.4) and of the
likelihood with a background term (Sect. 6).

* DS: the hat functions of the model grid sum to one, so every fine bin's
  column of DS sums to its width; linear interpolation reproduces linear
  functions, so sum_i E_i DS[i, e] is the integral of E over the bin for
  bins inside the model grid; each entry equals an adaptive quadrature of
  the hat function (scipy, independent of the exact splitting);
* response: a diagonal RMF gives RSP = DS diag(A); a response of fine
  bins that coincide with the model grid's cells integrates each cell's
  two hats to half its width;
* absorption: a transmission table sampled from exp(-N_ref s(E)) returns
  s(E) at its own nodes, and the transmission at N_H is the table value to
  the power N_H / N_ref;
* background: b = 0 is the plain Poisson likelihood (scipy.stats.poisson);
  with b the likelihood equals the plain one evaluated at m + b.
"""
import numpy as np
import pytest
from scipy import integrate, stats

from oracle import instrument as I


def grid():
    return np.geomspace(0.2, 3.0, 17)


def fine_bins(lo=0.12, hi=3.6, n=60):
    edges = np.sort(np.concatenate([np.geomspace(lo, hi, n + 1)]))
    return edges[:-1], edges[1:]


def test_ds_partition_of_unity_and_linear_reproduction():
    em = grid()
    lo, hi = fine_bins()
    ds = I.ds_matrix(em, lo, hi)
    assert np.allclose(ds.sum(axis=0), hi - lo, rtol=1e-13, atol=0)
    inside = (lo >= em[0]) & (hi <= em[-1])
    assert inside.sum() > 20
    first = em @ ds[:, inside]
    assert np.allclose(first, 0.5 * (hi[inside] ** 2 - lo[inside] ** 2), rtol=1e-12)


def test_ds_against_quadrature():
    em = grid()
    lo, hi = fine_bins(n=12)
    ds = I.ds_matrix(em, lo, hi)
    for i in (0, 5, 16):
        fp = np.zeros(em.size)
        fp[i] = 1.0
        for e in range(lo.size):
            q, _ = integrate.quad(lambda x: np.interp(x, em, fp), lo[e], hi[e], points=em[(em > lo[e]) & (em < hi[e])],
                                  epsabs=1e-14, epsrel=1e-12, limit=200)
            assert abs(ds[i, e] - q) <= 1e-12 * max(1.0, abs(q)) + 1e-15


def test_response_special_cases():
    em = grid()
    lo, hi = fine_bins(n=40)
    rng = np.random.default_rng(1)
    area = rng.uniform(50, 500, lo.size)
    rsp = I.response(em, lo, hi, area, np.eye(lo.size))
    assert np.allclose(rsp, I.ds_matrix(em, lo, hi) * area[None, :], rtol=1e-14)
    # fine bins equal to the model cells: each cell gives half its width to each end hat
    lo2, hi2 = em[:-1], em[1:]
    ds = I.ds_matrix(em, lo2, hi2)
    w = hi2 - lo2
    assert np.allclose(np.diag(ds[:-1]), 0.5 * w, rtol=1e-14)
    assert np.allclose(np.diag(ds[1:]), 0.5 * w, rtol=1e-14)
    assert np.count_nonzero(np.abs(ds) > 1e-300) == 2 * w.size


def test_absorption_table_power_scaling():
    e_tab = np.geomspace(0.1, 10.0, 200)
    nref = 4e18
    s_true = 2.4e-22 * e_tab ** -2.6
    att = np.exp(-nref * s_true)
    sig = I.sigma_from_table(e_tab, att, nref, e_tab)
    assert np.allclose(sig, s_true, rtol=1e-9)
    em = np.geomspace(0.2, 3.0, 33)
    nh = 2e19
    via_sigma = np.exp(-nh * I.sigma_from_table(e_tab, att, nref, em))
    assert np.allclose(via_sigma, np.interp(em, e_tab, att) ** (nh / nref), rtol=1e-12)


def test_background_likelihood():
    rng = np.random.default_rng(4)
    m = rng.uniform(0.1, 50, (8, 30))
    b = rng.uniform(0.0, 5.0, (8, 30))
    d = rng.poisson(m + b)
    assert np.isclose(I.loglike_with_background(m, np.zeros_like(m), d), stats.poisson.logpmf(d, m).sum(),
                      rtol=1e-12)
    assert np.isclose(I.loglike_with_background(m, b, d), stats.poisson.logpmf(d, m + b).sum(), rtol=1e-12)
    m0 = m.copy()
    m0[0, 0] = 0.0
    d0 = d.copy()
    d0[0, 0] = 3
    assert I.loglike_with_background(m0, np.zeros_like(m), d0) == -np.inf
    assert np.isfinite(I.loglike_with_background(m0, b + 0.5, d0))
