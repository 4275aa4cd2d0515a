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
