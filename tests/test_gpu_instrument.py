"""GPU checks of the instrument pipeline and the background term (Sects.
2.8.4, 7) through the C ABI, against the oracle.

* a response built by ``ppm_response_build`` from OGIP files written by the
  test helper, and an absorption cross-section from a transmission table
  (``ppm_sigma_from_table``), feed a plan whose counts match the oracle's
  forward model on the same arrays (1e-4 per bin above 1e-6 of the peak);
* with background counts the likelihood equals the oracle's likelihood of
  model plus background, the model counts are unchanged, an all-zero
  background is bit-identical to none;
* the gradient with background against the oracle's central differences of
  that likelihood (the gate of the gradient tests: 1e-5 relative, or twice
  the spread of the differences over steps 1e-5 .. 1e-7).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import instrument as I
import synthetic as syn
from fdcheck import fd_gate, report
from fits_writer import write_arf, write_rmf

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def rel_err(got, ref, floor=1e-6):
    sel = ref >= floor * ref.max()
    return float(np.max(np.abs(got[sel] - ref[sel]) / ref[sel])), int(sel.sum())


def instrument_spec(tmp_path, n_cells=16, n_phase=32, n_energy=64, n_chan=120):
    import paper_2510_07764_amd as ppm
    spec, p = syn.config1(n_cells=n_cells, n_phase=n_phase, n_energy=n_energy)
    edges = np.geomspace(0.15, 3.5, 301)
    lo, hi = edges[:-1], edges[1:]
    area = 400 * np.exp(-((np.log(0.5 * (lo + hi)) - 0.3) / 0.8) ** 2) + 20
    ch_edges = np.linspace(0.1, 3.8, n_chan + 1)
    cen = 0.5 * (ch_edges[:-1] + ch_edges[1:])
    m = np.exp(-0.5 * ((cen[None, :] - (0.5 * (lo + hi))[:, None]) / 0.08) ** 2)
    m[m < 1e-5] = 0.0
    m /= m.sum(axis=1, keepdims=True)
    pa, pr = os.path.join(tmp_path, "i.arf"), os.path.join(tmp_path, "i.rmf")
    write_arf(pa, lo, hi, area)
    write_rmf(pr, lo, hi, m, ch_edges[:-1], ch_edges[1:])
    alo, ahi, a = ppm.read_arf(pa)
    rlo, rhi, rm, _, _ = ppm.read_rmf(pr)
    spec["rsp"] = ppm.build_response(spec["energy"], rlo, rhi, a, rm)
    e_tab = np.geomspace(0.05, 10, 400)
    nref = 4e18
    att = np.exp(-nref * 2.4e-22 * e_tab ** -2.6)
    spec["sigma"] = ppm.sigma_from_table(e_tab, att, nref, spec["energy"])
    return spec, p


def test_response_from_ogip_files(torch_dev, tmp_path):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = instrument_spec(tmp_path)
    _, cnt, _ = oracle.forward(spec, p)
    plan = ppm.Plan(spec, max_batch=1)
    got = plan.forward(torch.tensor(p[None], dtype=torch.float64, device=dev)).cpu().numpy()[0]
    err, n = rel_err(got, cnt)
    print(f"OGIP response: counts max rel err {err:.3e} over {n} bins", flush=True)
    assert err < TOL


def test_background_likelihood(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=16, n_phase=32, n_energy=64)
    _, cnt, _ = oracle.forward(spec, p)
    rng = np.random.default_rng(8)
    bkg = rng.uniform(0.0, 0.5, cnt.shape) * cnt.mean()
    data = rng.poisson(cnt + bkg).astype(np.int32)
    dt = torch.tensor(data, device=dev)
    pt = torch.tensor(p[None], dtype=torch.float64, device=dev)
    plan0 = ppm.Plan(spec, max_batch=1)
    planb = ppm.Plan(dict(spec, background=bkg), max_batch=1)
    planz = ppm.Plan(dict(spec, background=np.zeros_like(bkg)), max_batch=1)
    c0, cb = torch.empty((1, 32, 300), dtype=torch.float64, device=dev), torch.empty((1, 32, 300), dtype=torch.float64, device=dev)
    l0 = plan0.loglike(pt, dt, counts=c0).item()
    lb = planb.loglike(pt, dt, counts=cb).item()
    lz = planz.loglike(pt, dt).item()
    assert torch.equal(c0, cb)                      # counts are the model's own
    assert lz == l0
    ref = I.loglike_with_background(cnt, bkg, data)
    assert abs(lb - ref) <= TOL * np.abs(data - cnt - bkg).sum()
    assert abs(lb - l0) > 1.0                       # the background matters here
    with pytest.raises(ppm.PPMError, match="background"):
        ppm.Plan(dict(spec, background=-bkg), max_batch=1)


def test_background_gradient(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=16, n_phase=32, n_energy=64)
    os_ = oracle.OracleSpec(spec)
    _, cnt, _ = oracle.forward(os_, p)
    rng = np.random.default_rng(9)
    bkg = rng.uniform(0.2, 1.0, cnt.shape) * cnt.mean()
    data = rng.poisson(cnt + bkg).astype(np.int32)
    q = syn.config4_draws(1)[0]

    def ll(x):
        _, c, _ = oracle.forward(os_, x)
        return I.loglike_with_background(c, bkg, data)

    # reference: the oracle's counts differenced over a ladder of steps and
    # contracted with d logL / d m = d / (m + b) - 1; true relative error
    # (no floor), bracketed by the differences at the kinked table
    fds = {s: oracle.fd_gradient_counts(os_, q, data, syn.GRAD_SLOTS, rel_step=s, background=bkg)
           for s in (3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7)}
    plan = ppm.Plan(dict(spec, background=bkg), max_batch=1, grad=True)
    lg, gg = plan.loglike_grad(torch.tensor(q[None], dtype=torch.float64, device=dev), torch.tensor(data, device=dev))
    g = gg.cpu().numpy()[0]
    rel, bound, delta = fd_gate(g, fds, kinked=True)
    report(g, fds, rel, bound, delta)
    assert np.all(rel <= bound)
    assert lg.item() == pytest.approx(ll(q), rel=1e-5)
