"""Pins of the oracle's parallel-tempered Metropolis sampler (Sect. 6).

* Philox4x32-10 against its published known-answer values (zero counter and
  key, all-ones counter and key, and the pi-digits counter and key);
* 53-bit uniforms in [0, 1) and uniform (chi-square), Box-Muller normals
  with the moments and Kolmogorov-Smirnov distance of N(0, 1);
* the sampler's stationary distributions on a correlated Gaussian target:
  the cold chain reproduces the target's mean and covariance, and the state
  at inverse temperature beta has covariance Sigma / beta (the target of a
  tempered level is likelihood^beta), with and without swaps; a single
  temperature reduces to plain random-walk Metropolis.
A wrong sign, index or factor in the proposal scaling, the acceptance or
the swap rule moves one of these by far more than its tolerance.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import sampler as S


@pytest.mark.parametrize("ctr,key,expect", [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(ctr, key, expect):
    out = S.philox4x32_10(np.array(ctr, dtype=np.uint64), key)
    assert [int(x) for x in out] == list(expect)


def test_uniforms_and_normals():
    u = S.uniforms(7, np.arange(200000), S.PURPOSE_ACCEPT, 12345)
    assert u.min() >= 0.0 and u.max() < 1.0
    hist, _ = np.histogram(u, bins=50, range=(0, 1))
    assert stats.chisquare(hist).pvalue > 1e-3
    z = S.normals(3, np.arange(50000), 2, 99).ravel()
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.02
    assert stats.kstest(z, "norm").statistic < 0.01
    # distinct purposes and steps give unrelated streams
    u2 = S.uniforms(8, np.arange(200000), S.PURPOSE_ACCEPT, 12345)
    assert abs(np.corrcoef(u, u2)[0, 1]) < 0.01


SIGMA = np.array([[1.0, 0.6], [0.6, 2.0]])
PREC = np.linalg.inv(SIGMA)


def gauss_logl(p):
    x = p[:, :2]
    return -0.5 * np.einsum("ni,ij,nj->n", x, PREC, x)


def run_all_levels(cfg, n_steps, burn):
    params = np.zeros((cfg.T, cfg.C, 16))
    logl = gauss_logl(params.reshape(-1, 16)).reshape(cfg.T, cfg.C)
    keep = []
    for n in range(n_steps):
        prop = S.propose(cfg, params, n)
        pl = gauss_logl(prop.reshape(-1, 16)).reshape(cfg.T, cfg.C)
        params, logl, _, _ = S.accept_and_swap(cfg, params, logl, prop, pl, n)
        if n >= burn:
            keep.append(params[:, :, :2].copy())
    return np.array(keep)    # [steps, T, C, 2]


@pytest.mark.parametrize("swap_every", [0, 1])
def test_tempered_gaussian_levels(swap_every):
    betas = [1.0, 0.5, 0.25]
    cfg = S.PTConfig(64, betas, [0, 1], [-50, -50], [50, 50], [1.2, 1.6], seed=2024, swap_every=swap_every)
    x = run_all_levels(cfg, 2500, 500)
    for t, b in enumerate(betas):
        s = x[:, t].reshape(-1, 2)
        assert np.all(np.abs(s.mean(axis=0)) < 0.12 / np.sqrt(b)), (t, s.mean(axis=0))
        cov = np.cov(s.T)
        assert np.allclose(cov * b, SIGMA, rtol=0.1, atol=0.06), (t, cov * b)


def test_single_temperature_is_metropolis_and_box_prior():
    cfg = S.PTConfig(128, [1.0], [0], [-1.0], [1.5], [0.8], seed=7, swap_every=0)
    chain, chain_l, n_acc, _, _, _ = S.run(cfg, np.zeros((1, 128, 16)),
                                           lambda p: -0.5 * p[:, 0] ** 2, 3000)
    s = chain[500:, :, 0].ravel()
    assert s.min() >= -1.0 and s.max() <= 1.5                 # the box is never left
    # target: N(0, 1) truncated to [-1, 1.5]
    a, b = -1.0, 1.5
    tm = stats.truncnorm(a, b)
    assert abs(s.mean() - tm.mean()) < 0.02 and abs(s.var() - tm.var()) < 0.02
    assert 0.2 < n_acc.sum() / (3000 * 128) < 0.9
