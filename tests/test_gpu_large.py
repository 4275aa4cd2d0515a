"""GPU parity at the full sizes of the stress workload and of the uneven-
resolution batch, against stored FP64 oracle counts (written by
tests/golden/make_golden_large.py, which calls only the oracle).

Bar as in the other parity tests: per phase-channel bin at or above 1e-6 of
the peak, |gpu - oracle| / oracle <= 1e-4.
"""
import json
import os

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def rel_err(got, ref, floor=1e-6):
    sel = ref >= floor * ref.max()
    return float(np.max(np.abs(got[sel] - ref[sel]) / ref[sel])), int(sel.sum())


def test_config2_full_size(torch_dev):
    """Compactness 0.28, a 1.2 rad cap straddling the pole and a 0.05 rad
    crescent near grazing at inclination 85 deg: 512x512 cells per spot,
    512 fine phases, 256 phases, 256 energies, 300 channels."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    ref = np.load(os.path.join(HERE, "golden", "config2_counts.npy"))
    meta = json.load(open(os.path.join(HERE, "golden", "large_meta.json")))["config2"]
    assert meta["diag"]["n_multi_image"] == 0
    spec, p = syn.config2()
    plan = ppm.Plan(spec, max_batch=1)
    pt = torch.tensor(p[None], dtype=torch.float64, device=dev)
    got = plan.forward(pt)
    torch.cuda.synchronize()
    got = got.cpu().numpy()[0]
    assert plan.status(1).cpu().numpy().tolist() == [0]
    err, n = rel_err(got, ref)
    print(f"config2 full: counts max rel err {err:.3e} over {n} bins; visible pairs "
          f"{plan.visible_pairs(1)} vs {meta['diag']['n_visible_pairs']}", flush=True)
    assert err < TOL
    assert plan.visible_pairs(1) == meta["diag"]["n_visible_pairs"]


def test_config3_sampled_instances_in_uneven_batch(torch_dev):
    """The first 24 seeded sampler draws with their own grids (64, 128, 256
    or 512 cells per side) in one batched call; the first draw of each of
    the resolutions 64, 128 and 256 against its stored oracle counts, and
    every instance finite with status 0."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    stored = np.load(os.path.join(HERE, "golden", "config3_counts.npz"))
    draws, res = syn.config3_draws()
    B = 24
    picks = {}
    for i, n in enumerate(res):
        if int(n) in (64, 128, 256) and int(n) not in picks:
            picks[int(n)] = i
    assert max(picks.values()) < B
    nc = np.ascontiguousarray(res[:B], dtype=np.int32)
    assert len(set(nc.tolist())) >= 3
    spec, _ = syn.config1()
    plan = ppm.Plan(spec, max_batch=B, max_cells=int(nc.max()))
    pt = torch.tensor(draws[:B], dtype=torch.float64, device=dev)
    got = plan.forward(pt, n_cells=nc)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.all(plan.status(B).cpu().numpy() == 0)
    for n, i in sorted(picks.items()):
        ref = stored["res%d" % n]
        err, nb = rel_err(got[i], ref)
        print(f"config3 draw {i} at {n}x{n}: counts max rel err {err:.3e} over {nb} bins", flush=True)
        assert err < TOL, (n, i, err)
    # the first draw at 512x512 cells (stored by make_golden_flux.py)
    if "res512" not in stored.files:
        pytest.skip("stored 512x512 oracle counts not generated yet (tests/golden/make_golden_flux.py)")
    i512 = json.load(open(os.path.join(HERE, "golden", "large_meta.json")))["config3_res512"]["index"]
    assert i512 < B and nc[i512] == 512
    err, nb = rel_err(got[i512], stored["res512"])
    print(f"config3 draw {i512} at 512x512: counts max rel err {err:.3e} over {nb} bins", flush=True)
    assert err < TOL


def test_uneven_batch_of_1024_equals_single_calls(torch_dev):
    """The 1024 seeded sampler draws with their own grids (64..512 cells per
    side) in one call, with one ring per group and with groups of four: the
    instances checked (the first draw at each resolution, and draws spread
    over the batch) equal their single calls bit for bit, every instance is
    valid and its counts finite."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    draws, res = syn.config3_draws()
    B = len(draws)
    nc = np.ascontiguousarray(res, dtype=np.int32)
    spec, _ = syn.config1()
    plan = ppm.Plan(spec, max_batch=B, max_cells=512)
    pt = torch.tensor(draws, dtype=torch.float64, device=dev)
    check = sorted({int(np.argmax(res == n)) for n in (64, 128, 256, 512)} | {1, 333, 517, 768, B - 1})
    for G in (1, 4):
        plan.set_tiles(phase_tile=128, ring_group=G)
        got = plan.forward(pt, n_cells=nc)
        torch.cuda.synchronize()
        print(f"ring group {G}: {B} instances in {plan.passes} workspace passes", flush=True)
        got = got.cpu().numpy()
        assert np.all(np.isfinite(got)) and np.all(plan.status(B).cpu().numpy() == 0)
        for i in check:
            one = plan.forward(pt[i:i + 1].contiguous(), n_cells=nc[i:i + 1]).cpu().numpy()[0]
            assert np.array_equal(one, got[i]), (G, i, int(nc[i]))


def flux_bins_err(got, ref, floor=1e-6):
    sel = ref >= floor * ref.max()
    return float(np.max(np.abs(got[sel] - ref[sel]) / ref[sel])), int(sel.sum())


@pytest.mark.parametrize("which", ["config1", "config2"])
def test_full_size_flux_per_bin(torch_dev, which):
    """Photon flux before absorption and response (F_t of Eq. 47) at full
    size, per (phase, energy) bin against the stored oracle flux: the bar is
    checked before the 300-channel fold averages over neighbouring
    energies."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    path = os.path.join(HERE, "golden", f"{which}_flux.npy")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle flux not generated yet: {path} (tests/golden/make_golden_flux.py)")
    ref = np.load(path)
    spec, p = syn.config1() if which == "config1" else syn.config2()
    plan = ppm.Plan(spec, max_batch=1)
    got = plan.flux(torch.tensor(p[None], dtype=torch.float64, device=dev)).cpu().numpy()[0]
    err, nb = flux_bins_err(got, ref)
    print(f"{which} full-size flux: max rel err {err:.3e} over {nb} (phase, energy) bins", flush=True)
    assert err < TOL


def test_resolution_tier_512_against_oracle_1024(torch_dev):
    """Discretisation error of the 512x512 surface grid (the resolution tiers
    of Sect. 5): the GPU flux of the stress workload at 512x512 cells per
    spot against the FP64 oracle at 1024x1024 (everything else at full
    size).  Reported, not a parity bar: the difference measures the surface
    grid, not the implementation.  The assertion only guards against a
    gross error (ten times the measured figures, ~1e-4 per bin)."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    path = os.path.join(HERE, "golden", "config2_1024_flux.npy")
    if not os.path.exists(path):
        pytest.skip(f"stored oracle flux not generated yet: {path} (tests/golden/make_golden_res.py)")
    ref = np.load(path)
    spec, p = syn.config2()
    plan = ppm.Plan(spec, max_batch=1)
    got = plan.flux(torch.tensor(p[None], dtype=torch.float64, device=dev)).cpu().numpy()[0]
    sel = ref >= 1e-6 * ref.max()
    r = np.abs(got[sel] - ref[sel]) / ref[sel]
    tot = abs(got.sum() - ref.sum()) / ref.sum()
    print(f"config2 GPU 512x512 vs oracle 1024x1024 flux: max rel {r.max():.3e}, median {np.median(r):.3e}, "
          f"99th percentile {np.quantile(r, 0.99):.3e} over {int(sel.sum())} bins; total {tot:.3e}", flush=True)
    assert r.max() < 1e-3
