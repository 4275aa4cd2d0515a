"""GPU checks of the ring groups of the windowed accumulation kernel
(``ppm_tiles.ring_group``): a work-group sums up to G consecutive rings of
one instance into one FP32 partial spectrum per phase, and the ring
reduction adds the groups in FP64 (Eq. 47).

Bars: each group size against the FP64 oracle at the parity bar (1e-4 per
bin above 1e-6 of the peak); for a fixed group size, bit-for-bit
reproducibility, batch = single calls, independence of the phase tile,
workspace passes and graph replays; across group sizes agreement to the
FP32 rounding of the group sums (1e-5 relative per bin here).
"""
import numpy as np
import pytest

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def rel_err(got, ref, floor=1e-6):
    sel = ref >= floor * ref.max()
    return float(np.max(np.abs(got[sel] - ref[sel]) / ref[sel]))


def test_group_sizes_against_oracle_and_each_other(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=20, n_phase=24, n_energy=128)
    _, cnt, _ = oracle.forward(spec, p)
    plan = ppm.Plan(spec, max_batch=1)
    assert plan.ring_group == 1
    pt = torch.tensor(p[None], dtype=torch.float64, device=dev)
    ref = None
    for G in (1, 2, 3, 7, 16, 40, 64):
        plan.set_tiles(ring_group=G)
        a = plan.forward(pt).cpu().numpy()[0]
        b = plan.forward(pt).cpu().numpy()[0]
        assert np.array_equal(a, b), G
        err = rel_err(a, cnt)
        print(f"ring group {G}: counts vs oracle {err:.3e}", flush=True)
        assert err < TOL
        if ref is None:
            ref = a
        else:
            assert rel_err(a, ref) < 1e-5
        for t in (5, 24):
            plan.set_tiles(phase_tile=t)
            assert np.array_equal(plan.forward(pt).cpu().numpy()[0], a), (G, t)
        plan.set_tiles(phase_tile=8)
    with pytest.raises(ppm.PPMError, match="ring_group"):
        plan.set_tiles(ring_group=65)
    with pytest.raises(ppm.PPMError, match="ring_group"):
        plan.set_tiles(ring_group=0)


def test_group_batch_equals_singles_uneven_grids(torch_dev):
    """An uneven batch (per-instance grids, some rings hidden) with groups of
    5: each instance equals its single call bit for bit, also when the batch
    runs in several workspace passes."""
    import os
    import subprocess
    import sys
    import json
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, _ = syn.config1(n_cells=16, n_phase=16, n_energy=64)
    draws, _ = syn.config3_draws(6)
    nc = np.array([8, 16, 4, 12, 16, 6], dtype=np.int32)
    plan = ppm.Plan(spec, max_batch=6, max_cells=16)
    plan.set_tiles(ring_group=5)
    pt = torch.tensor(draws, dtype=torch.float64, device=dev)
    batch = plan.forward(pt, n_cells=nc).cpu().numpy()
    for i in range(6):
        one = plan.forward(pt[i:i + 1].contiguous(), n_cells=nc[i:i + 1]).cpu().numpy()[0]
        assert np.array_equal(one, batch[i]), i
    code = r'''
import os, sys, json
sys.path.insert(0, os.getcwd())
import numpy as np, torch
import synthetic as syn, paper_2510_07764_amd as ppm
spec, _ = syn.config1(n_cells=16, n_phase=16, n_energy=64)
draws, _ = syn.config3_draws(6)
nc = np.array([8, 16, 4, 12, 16, 6], dtype=np.int32)
plan = ppm.Plan(spec, max_batch=6, max_cells=16)
plan.set_tiles(ring_group=5)
out = plan.forward(torch.tensor(draws, dtype=torch.float64, device="cuda"), n_cells=nc)
print(json.dumps(out.cpu().numpy().tolist()))
'''
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PPM_MAX_CHUNK="2")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=root, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert np.array_equal(np.array(json.loads(out.stdout.strip().splitlines()[-1])), batch)


def test_group_flux_and_loglike_paths(torch_dev):
    """Flux before absorption and the likelihood with groups of 8 against the
    oracle, and the gradient plan's forward (which keeps that flux) with a
    group size set: logL of the gradient call equals ppm_loglike's."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=16, n_phase=20, n_energy=64)
    ft, cnt, _ = oracle.forward(spec, p)
    data = syn.poisson_data(cnt)
    plan = ppm.Plan(spec, max_batch=1, grad=True)
    plan.set_tiles(ring_group=8)
    pt = torch.tensor(p[None], dtype=torch.float64, device=dev)
    assert rel_err(plan.flux(pt).cpu().numpy()[0], ft) < TOL
    dt = torch.tensor(data, device=dev)
    ll = plan.loglike(pt, dt)
    ll2, _ = plan.loglike_grad(pt, dt)
    assert torch.equal(ll, ll2)
    assert ll.item() == pytest.approx(oracle.loglike_from_counts(cnt, data), rel=1e-6)


def test_autotuner_reports_ring_groups(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, _ = syn.config1(n_cells=8, n_phase=16, n_energy=64)
    q = torch.tensor(syn.config4_draws(4), dtype=torch.float64, device=dev)
    plan = ppm.Plan(spec, max_batch=4)
    rep = plan.autotune(q, reps=3)
    print(rep, flush=True)
    assert sorted(rep["group"]) == [1, 2, 4, 8, 16]
    assert plan.ring_group == rep["ring_group"] == min(rep["group"], key=rep["group"].get)
