"""GPU parity of the adjoint (``ppm_loglike_grad``, through the C ABI)
against central finite differences of the FP64 CPU oracle.

The gradient is d logL / d(M, R_e, i, Phi, N_H, theta_1, zeta_1, logT_1,
theta_2, zeta_2, logT_2, dphi_2), evaluated away from the data's truth
(the first seeded draw within +-5% of the config-1 parameters) so that no
component vanishes by construction.

Bar, per component n: |g_gpu - FD_n(1e-6)| <= max(1e-5 * max(|FD_n|, 1e-3 *
max|FD|), 2 * spread_n), where FD_n(s) is the oracle's central difference
with step s * |theta_n| and spread_n = max - min of FD_n over s in {1e-5,
1e-6, 1e-7}: the model is piecewise polynomial (linear phase interpolation,
piecewise-cubic Lagrange stencils), so central differences converge only
as far as their steps avoid stencil kinks, and the spread measures how far
that is.  Where the differences have converged the bar is 1e-5 relative.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
NAMES = ("M", "R_e", "i", "Phi", "N_H", "theta1", "zeta1", "logT1", "theta2", "zeta2", "logT2", "dphi2")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def fd_gate(g, fds):
    """fds: {step: FD vector}; returns per-component (error, bound)."""
    f6 = fds[1e-6]
    spread = np.max([fds[s] for s in fds], axis=0) - np.min([fds[s] for s in fds], axis=0)
    floor = 1e-3 * np.abs(f6).max()
    bound = np.maximum(1e-5 * np.maximum(np.abs(f6), floor), 2.0 * spread)
    return np.abs(g - f6), bound


def small_problem(cells, phases, energies):
    spec, p = syn.config1(n_cells=cells, n_phase=phases, n_energy=energies)
    os_ = oracle.OracleSpec(spec)
    _, cnt, _ = oracle.forward(os_, p)
    data = syn.poisson_data(cnt)
    q = syn.config4_draws(1)[0]
    return spec, os_, data, q


@pytest.mark.parametrize("cells,phases,energies", [(16, 32, 64), (24, 40, 256)])
def test_grad_vs_oracle_fd(torch_dev, cells, phases, energies):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, os_, data, q = small_problem(cells, phases, energies)
    fds = {s: oracle.fd_gradient(os_, q, data, syn.GRAD_SLOTS, rel_step=s) for s in (1e-5, 1e-6, 1e-7)}
    fd4 = oracle.fd_gradient(os_, q, data, syn.GRAD_SLOTS, rel_step=1e-4)
    plan = ppm.Plan(spec, max_batch=1, grad=True)
    ll, g = plan.loglike_grad(torch.tensor(q[None], dtype=torch.float64, device=dev),
                              torch.tensor(data, device=dev))
    g = g.cpu().numpy()[0]
    err, bound = fd_gate(g, fds)
    floor = 1e-3 * np.abs(fds[1e-6]).max()
    for n in range(12):
        print("%-7s gpu %+.9e  fd(1e-6) %+.9e  err/scale %.1e  bound/scale %.1e  |gpu-fd(1e-4)|/scale %.1e"
              % (NAMES[n], g[n], fds[1e-6][n], err[n] / max(abs(fds[1e-6][n]), floor),
                 bound[n] / max(abs(fds[1e-6][n]), floor), abs(g[n] - fd4[n]) / max(abs(fd4[n]), floor)))
    assert np.all(err <= bound), [(NAMES[n], err[n], bound[n]) for n in range(12) if err[n] > bound[n]]
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
    fds = {float(k[3:]): np.array(v) for k, v in gold.items() if k.startswith("fd_")}
    steps = sorted(s for s in fds if s <= 1e-5) or [1e-6]
    sub = {s: fds[s] for s in steps}
    sub.setdefault(1e-6, fds[1e-6])
    err, bound = fd_gate(g, sub)
    floor = 1e-3 * np.abs(fds[1e-6]).max()
    for n in range(12):
        print("%-7s gpu %+.9e  fd(1e-6) %+.9e  err/scale %.1e  |gpu-fd(1e-4)|/scale %.1e"
              % (NAMES[n], g[n], fds[1e-6][n], err[n] / max(abs(fds[1e-6][n]), floor),
                 abs(g[n] - fds[1e-4][n]) / max(abs(fds[1e-4][n]), floor)))
    assert ll.item() == pytest.approx(gold["loglike"], rel=1e-6)
    assert np.all(err <= bound), [(NAMES[n], err[n], bound[n]) for n in range(12) if err[n] > bound[n]]
