"""GPU checks of the launch shape of the accumulation kernels and of the
autotuner that picks it (``ppm_set_tiles`` / ``ppm_autotune``, through the
C ABI).

The forward model is independent of the phase tile by construction: each
phase's sum over cells and energies runs in one wave in the same order
whatever the tile, so counts must agree bit for bit across tiles.  The
adjoint's per-block partial sums are regrouped by the tile, so gradients
agree to rounding (1e-11 relative here).  One tile setting is also checked
against the FP64 oracle at the same bar as the parity tests (1e-4 per bin
above 1e-6 of the peak).
"""
import numpy as np
import pytest

import oracle
import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def _counts(plan, torch, dev, params, n_cells=None):
    out = plan.forward(torch.tensor(params, dtype=torch.float64, device=dev), n_cells=n_cells)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("which", ["table", "table_cubic", "blackbody"])
def test_forward_bitwise_independent_of_phase_tile(torch_dev, which):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    if which == "blackbody":
        spec, p = syn.config0()
        spec = dict(spec, n_phase=40)
    else:
        # 40 phases: ragged last tile for every tile size except 1, 4, 8, 40
        spec, p = syn.config1(n_cells=24, n_phase=40, n_energy=256)
        if which == "table_cubic":
            spec = dict(spec, interp=ppm.INTERP_CUBIC)
    plan = ppm.Plan(spec, max_batch=2)
    params = np.stack([p, syn.config4_draws(1)[0] if which != "blackbody" else p])
    assert plan.tiles == (8, 8)
    ref = _counts(plan, torch, dev, params)
    for t in (1, 3, 4, 5, 12, 16, 24, 32, 40, 64, 256):
        plan.set_tiles(phase_tile=t)
        assert plan.tiles[0] == t
        got = _counts(plan, torch, dev, params)
        assert np.array_equal(got, ref), (which, t, np.max(np.abs(got - ref)))
    if which == "table":
        _, cnt, _ = oracle.forward(oracle.OracleSpec(spec), p)
        sel = cnt >= 1e-6 * cnt.max()
        err = np.max(np.abs(ref[0][sel] - cnt[sel]) / cnt[sel])
        print(f"tile-independent counts vs oracle: max rel err {err:.3e}", flush=True)
        assert err < 1e-4


def test_forward_tiles_with_uneven_grids(torch_dev):
    """Per-instance grids (work list sorted by size) with several tiles."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, _ = syn.config1(n_cells=16, n_phase=24, n_energy=64)
    draws, _ = syn.config3_draws(5)
    nc = np.array([8, 16, 4, 12, 16], dtype=np.int32)
    plan = ppm.Plan(spec, max_batch=5, max_cells=16)
    ref = _counts(plan, torch, dev, draws, n_cells=nc)
    for t in (4, 16, 24):
        plan.set_tiles(phase_tile=t)
        assert np.array_equal(_counts(plan, torch, dev, draws, n_cells=nc), ref), t


def test_gradient_across_adjoint_tiles(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=16, n_phase=40, n_energy=64)
    _, cnt, _ = oracle.forward(oracle.OracleSpec(spec), p)
    data = torch.tensor(syn.poisson_data(cnt), device=dev)
    q = torch.tensor(syn.config4_draws(3), dtype=torch.float64, device=dev)
    plan = ppm.Plan(spec, max_batch=3, grad=True)
    ll0, g0 = plan.loglike_grad(q, data)
    ll0, g0 = ll0.cpu().numpy(), g0.cpu().numpy()
    scale = np.maximum(np.abs(g0), 1e-3 * np.abs(g0).max(axis=1, keepdims=True))
    for fwd, adj in ((8, 16), (4, 24), (16, 40), (32, 8), (8, 256)):
        plan.set_tiles(phase_tile=fwd, phase_tile_grad=adj)
        ll, g = plan.loglike_grad(q, data)
        ll, g = ll.cpu().numpy(), g.cpu().numpy()
        assert np.array_equal(ll, ll0), (fwd, adj)   # forward and likelihood do not regroup
        err = np.max(np.abs(g - g0) / scale)
        assert err < 1e-11, (fwd, adj, err)


def test_split_launches_bit_identical(torch_dev):
    """An accumulation launch is split over sub-ranges of the work list when
    its grid would pass the 2^32-thread launch limit (a batch of 1,024
    workload-1 vectors at phase tile 4).  Forced here on a small batch by
    lowering the limit (PPM_MAX_LAUNCH_THREADS): forward counts, logL and the
    gradient, and a temperature-map forward, are bit-identical to the
    unsplit launches (every block writes only its own ring's outputs)."""
    import os
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=16, n_phase=32, n_energy=64)
    _, cnt, _ = oracle.forward(oracle.OracleSpec(spec), p)
    data = torch.tensor(syn.poisson_data(cnt), device=dev)
    q = torch.tensor(syn.config4_draws(4), dtype=torch.float64, device=dev)
    plan = ppm.Plan(spec, max_batch=4, grad=True)
    plan.set_tiles(phase_tile=4, phase_tile_grad=8)
    mspec, mp, mm = syn.map_config(4, "full", n_phase=32, n_energy=64)
    mplan = ppm.Plan(mspec, max_batch=2)
    mpt = torch.tensor(np.stack([mp, mp]), dtype=torch.float64, device=dev)
    mpt[1, 3] = 0.25
    mmt = torch.tensor(np.stack([mm, mm[::-1].copy()]), dtype=torch.float64, device=dev)

    def run():
        c = plan.forward(q).cpu().numpy()
        ll, g = plan.loglike_grad(q, data)
        mc = mplan.forward_map(mpt, mmt).cpu().numpy()
        torch.cuda.synchronize()
        return c, ll.cpu().numpy(), g.cpu().numpy(), mc

    ref = run()
    # 8 work-list entries per forward launch (8 tiles x 768 threads each)
    os.environ["PPM_MAX_LAUNCH_THREADS"] = str(8 * 8 * 768)
    try:
        got = run()
    finally:
        del os.environ["PPM_MAX_LAUNCH_THREADS"]
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_set_tiles_rejects_out_of_range(torch_dev):
    import paper_2510_07764_amd as ppm
    spec, _ = syn.config1(n_cells=8, n_phase=16, n_energy=32)
    plan = ppm.Plan(spec, max_batch=1, grad=True)
    plan.set_tiles(12, 16)
    for bad in ((0, 16), (257, 16), (12, 7), (12, 257)):
        with pytest.raises(ppm.PPMError, match="must lie in"):
            plan.set_tiles(*bad)
        assert plan.tiles == (12, 16)


def test_autotune_picks_a_candidate_and_keeps_results(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=32, n_phase=32, n_energy=256)
    _, cnt, _ = oracle.forward(oracle.OracleSpec(spec), p)
    data = torch.tensor(syn.poisson_data(cnt), device=dev)
    q = torch.tensor(syn.config4_draws(4), dtype=torch.float64, device=dev)
    plan = ppm.Plan(spec, max_batch=4, grad=True)
    ref = plan.forward(q).cpu().numpy()
    rep = plan.autotune(q, reps=3)
    print("autotune report:", rep, flush=True)
    # 32 phases: candidates 4, 8, 12, 16, 20, 24, 28, 32, 48, 64, 96, 128 give 8, 4, 3, 2, 2, 2, 2,
    # 1, 1, 1, 1, 1 tiles; those repeating a smaller candidate's count are dropped
    assert sorted(rep["forward"]) == [4, 8, 12, 16, 32]
    assert sorted(rep["grad"]) == [8, 16, 32]
    assert all(v > 0 for v in rep["forward"].values()) and all(v > 0 for v in rep["grad"].values())
    fwd, adj = rep["chosen"]
    assert rep["forward"][fwd] == min(rep["forward"].values())
    assert rep["grad"][adj] == min(rep["grad"].values())
    assert plan.tiles == (fwd, adj)
    G = rep["ring_group"]
    assert rep["group"][G] == min(rep["group"].values()) and plan.ring_group == G
    # results depend on the ring group only (at the FP32 rounding of the group sums)
    fresh = ppm.Plan(spec, max_batch=4, grad=True)
    fresh.set_tiles(ring_group=G)
    assert np.array_equal(plan.forward(q).cpu().numpy(), fresh.forward(q).cpu().numpy())
    if G == 1:
        assert np.array_equal(plan.forward(q).cpu().numpy(), ref)
    ll, g = plan.loglike_grad(q, data)
    assert np.all(np.isfinite(g.cpu().numpy()))


def test_graph_keeps_its_captured_tiles(torch_dev):
    """A HIP graph records the launch shape at capture; changing the plan's
    tiles afterwards leaves the graph's results unchanged."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=16, n_phase=32, n_energy=64)
    _, cnt, _ = oracle.forward(oracle.OracleSpec(spec), p)
    data = torch.tensor(syn.poisson_data(cnt), device=dev)
    q = torch.tensor(syn.config4_draws(2), dtype=torch.float64, device=dev)
    plan = ppm.Plan(spec, max_batch=2)
    eager = plan.loglike(q, data).cpu().numpy()
    g = ppm.GraphedLogLike(plan, data, 2)
    plan.set_tiles(phase_tile=32)
    for _ in range(3):
        out = g(q).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(out, eager)
    assert np.array_equal(plan.loglike(q, data).cpu().numpy(), eager)
