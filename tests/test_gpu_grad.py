"""GPU parity of the adjoint (``ppm_loglike_grad``, through the C ABI)
against central finite differences of the FP64 CPU oracle.

The gradient is d logL / d(M, R_e, i, Phi, N_H, theta_1, zeta_1, logT_1,
theta_2, zeta_2, logT_2, dphi_2), evaluated away from the data's truth
(the first seeded draw within +-5% of the config-1 parameters) so that no
component vanishes by construction.

Reference: the oracle's counts differenced centrally with steps
h_n = s |theta_n| over a ladder of s and contracted with the closed-form
d logL / d m (``oracle.fd_gradient_counts``).  The model is piecewise
polynomial (linear phase interpolation, piecewise-cubic Lagrange stencils
in mu and x, bilinear in logT / log g), so a difference converges only
while its step crosses no stencil or fine-phase kink.  Per component the
reference is the mean of the two adjacent ladder steps that agree best, and
their relative disagreement delta_n says how well the reference is known.

Bar, per component, on the true relative error (no floor).  On the
multilinear synthetic table (interpolation exact, no stencil kinks) every
component's differences converge to delta_n <= 1e-6 and the bar is
|g_n - FD_n| <= (1e-5 + delta_n) |FD_n|: 1e-5 relative for all twelve
components, Phi and dphi_2 included.  On the synthetic NSX-like table the
piecewise-cubic stencils put kinks inside every step for the phase-like
directions (Phi, dphi_2), whose differences wander by up to ~1e-4 between
steps; there the differences over the steps <= 1e-5 bracket the
derivative and the bar is 1e-5 beyond that bracket (printed per component).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synthetic as syn
from fdcheck import LADDER, NAMES, fd_gate, report

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def small_problem(cells, phases, energies, table="synthetic"):
    spec, p = syn.config1(n_cells=cells, n_phase=phases, n_energy=energies)
    if table == "multilinear":
        logi, axes = syn.atmosphere_table_multilinear()
        spec["atmos_logI"], spec["atmos_axes"] = logi, axes
    os_ = oracle.OracleSpec(spec)
    _, cnt, _ = oracle.forward(os_, p)
    data = syn.poisson_data(cnt)
    q = syn.config4_draws(1)[0]
    return spec, os_, data, q


@pytest.mark.parametrize("cells,phases,energies,table", [(8, 16, 32, "multilinear"), (16, 32, 64, "multilinear"),
                                                         (16, 32, 64, "synthetic"), (24, 40, 256, "synthetic")])
def test_grad_vs_oracle_fd(torch_dev, cells, phases, energies, table):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, os_, data, q = small_problem(cells, phases, energies, table)
    ladder = LADDER if cells <= 16 else LADDER[2:7]
    fds = {s: oracle.fd_gradient_counts(os_, q, data, syn.GRAD_SLOTS, rel_step=s) for s in ladder}
    plan = ppm.Plan(spec, max_batch=1, grad=True)
    ll, g = plan.loglike_grad(torch.tensor(q[None], dtype=torch.float64, device=dev),
                              torch.tensor(data, device=dev))
    g = g.cpu().numpy()[0]
    rel, bound, delta = fd_gate(g, fds, kinked=table != "multilinear")
    report(g, fds, rel, bound, delta)
    if table == "multilinear":
        # no stencil kinks: every component's reference is known to 1e-6
        assert np.all(delta <= 1e-6), [(NAMES[n], delta[n]) for n in range(12) if delta[n] > 1e-6]
    assert np.all(rel <= bound), [(NAMES[n], rel[n], bound[n]) for n in range(12) if rel[n] > bound[n]]
    # the likelihood value itself is the plain path's
    assert ll.item() == pytest.approx(oracle.loglike(os_, q, data), rel=1e-5)


def test_grad_logl_batch_determinism_autograd(torch_dev):
    """logL of the gradient call equals ppm_loglike bit for bit; a batch
    equals its single calls and repeats bit for bit; the autograd wrapper
    returns the adjoint in the twelve slots and zero elsewhere."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, os_, data, _ = small_problem(16, 32, 64)
    draws = syn.config4_draws(3)
    dt = torch.tensor(data, device=dev)
    plan = ppm.Plan(spec, max_batch=3, grad=True)
    pt = torch.tensor(draws, dtype=torch.float64, device=dev)
    ll, g = plan.loglike_grad(pt, dt)
    ll_plain = plan.loglike(pt, dt)
    assert torch.equal(ll, ll_plain)
    ll2, g2 = plan.loglike_grad(pt, dt)
    assert torch.equal(g, g2) and torch.equal(ll, ll2)
    for i in range(3):
        l1, g1 = plan.loglike_grad(pt[i:i + 1].contiguous(), dt)
        assert torch.equal(g1[0], g[i]) and torch.equal(l1[0], ll[i])
    p = pt.clone().requires_grad_(True)
    ppm.loglike_autograd(p, plan, dt).sum().backward()
    full = torch.zeros_like(pt)
    full[:, list(ppm.GRAD_SLOTS)] = g
    assert torch.equal(p.grad, full)
    # weighted backward
    p2 = pt.clone().requires_grad_(True)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device=dev)
    (ppm.loglike_autograd(p2, plan, dt) * w).sum().backward()
    assert torch.allclose(p2.grad, w[:, None] * full, rtol=0, atol=0)


def test_grad_invalid_instance_and_plan_errors(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, os_, data, q = small_problem(8, 16, 32)
    dt = torch.tensor(data, device=dev)
    bad = q.copy()
    bad[9] = -0.1                      # negative spot radius
    plan = ppm.Plan(spec, max_batch=2, grad=True)
    ll, g = plan.loglike_grad(torch.tensor(np.stack([q, bad]), dtype=torch.float64, device=dev), dt)
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    assert np.isfinite(ll[0]) and np.all(np.isfinite(g[0]))
    assert ll[1] == -np.inf and np.all(np.isnan(g[1]))
    assert plan.status(2).cpu().numpy().tolist() == [0, 4]
    fwd_only = ppm.Plan(spec, max_batch=1)
    with pytest.raises(ppm.PPMError, match="grad"):
        fwd_only.loglike_grad(torch.tensor(q[None], dtype=torch.float64, device=dev), dt)


def test_grad_multi_pass_and_graph(torch_dev):
    """Batches split over several workspace passes give the single-pass
    gradient bit for bit; a captured gradient evaluation replays exactly."""
    import subprocess
    import sys
    code = r'''
import os, sys, json
sys.path.insert(0, os.getcwd())
import numpy as np, torch
import oracle, synthetic as syn, paper_2510_07764_amd as ppm
spec, p = syn.config1(n_cells=8, n_phase=16, n_energy=32)
_, cnt, _ = oracle.forward(spec, p)
dt = torch.tensor(syn.poisson_data(cnt), device="cuda")
draws = syn.config4_draws(5)
pt = torch.tensor(draws, dtype=torch.float64, device="cuda")
plan = ppm.Plan(spec, max_batch=5, grad=True)
ll, g = plan.loglike_grad(pt, dt)
print(json.dumps({"ll": ll.cpu().numpy().tolist(), "g": g.cpu().numpy().tolist()}))
'''
    root = os.path.dirname(HERE)
    runs = []
    for chunk in ("2", "0"):
        env = dict(os.environ, PPM_MAX_CHUNK=chunk)
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=root,
                             timeout=300)
        assert out.returncode == 0, out.stderr[-2000:]
        runs.append(json.loads(out.stdout.strip().splitlines()[-1]))
    assert runs[0] == runs[1]
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, os_, data, _ = small_problem(8, 16, 32)
    dt = torch.tensor(data, device=dev)
    plan = ppm.Plan(spec, max_batch=2, grad=True)
    gl = ppm.GraphedLogLike(plan, dt, 2, grad=True)
    draws = syn.config4_draws(4)
    for rep in range(3):
        rows = torch.tensor(draws[rep % 2 * 2:rep % 2 * 2 + 2], dtype=torch.float64, device=dev)
        l1, g1 = gl(rows)
        l1, g1 = l1.clone(), g1.clone()
        torch.cuda.synchronize()
        l2, g2 = plan.loglike_grad(rows, dt)
        torch.cuda.synchronize()
        assert torch.equal(l1, l2) and torch.equal(g1, g2), rep


def test_grad_full_size_golden(torch_dev):
    """Config-1 size (128x128 cells per spot, 128 phases, 256 energies)
    against the stored oracle finite differences."""
    path = os.path.join(HERE, "golden", "config4_grad.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle gradient not generated")
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    with open(path) as f:
        gold = json.load(f)
    spec, _ = syn.config1()
    data = np.load(os.path.join(HERE, "golden", "config1_data.npy"))
    q = np.array(gold["params"])
    plan = ppm.Plan(spec, max_batch=1, grad=True)
    ll, g = plan.loglike_grad(torch.tensor(q[None], dtype=torch.float64, device=dev),
                              torch.tensor(data, device=dev))
    g = g.cpu().numpy()[0]
    fds = {float(k[4:]): np.array(v) for k, v in gold.items() if k.startswith("fdc_")}
    assert len(fds) >= 3, "stored chain-rule differences missing (tests/golden/make_golden_grad.py)"
    rel, bound, delta = fd_gate(g, fds, kinked=True)
    report(g, fds, rel, bound, delta)
    fd4 = np.array(gold["fd_0.0001"])
    print("vs the logL difference at step 1e-4:", np.round(np.abs(g - fd4) / np.abs(fd4), 7).tolist(), flush=True)
    assert ll.item() == pytest.approx(gold["loglike"], rel=1e-6)
    assert np.all(rel <= bound), [(NAMES[n], rel[n], bound[n]) for n in range(12) if rel[n] > bound[n]]
