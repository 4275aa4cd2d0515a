"""The allocation-free likelihood entry point (``ppm_loglike_noalloc``,
through the C ABI) against ``ppm_loglike`` on the same plan: the same
kernels, tiles and ring group, so logL and the model counts must agree bit
for bit, on two calls in a row (the second with a smaller batch, in the
static scratch the first call left behind), with and without a counts
buffer, and after calls of the regular entry point; a batch beyond the
64 MiB scratch is refused."""
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


def test_noalloc_equals_loglike(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=24, n_phase=32, n_energy=64)
    _, cnt, _ = oracle.forward(spec, p)
    dt = torch.tensor(syn.poisson_data(cnt), device=dev)
    draws = syn.config4_draws(3)
    plan = ppm.Plan(spec, max_batch=3)
    for G in (1, 4):
        plan.set_tiles(ring_group=G)
        for B in (3, 1):                                   # second call smaller
            pt = torch.tensor(draws[:B], dtype=torch.float64, device=dev)
            c1 = torch.empty((B, plan.n_phase, plan.n_chan), dtype=torch.float64, device=dev)
            c2 = torch.empty_like(c1)
            l1 = plan.loglike(pt, dt, counts=c1)
            l2 = plan.loglike_noalloc(pt, dt, counts=c2)
            l3 = plan.loglike_noalloc(pt, dt)
            torch.cuda.synchronize()
            print(f"G {G} B {B}: logL {l1.cpu().numpy()} noalloc {l2.cpu().numpy()}", flush=True)
            assert torch.equal(l1, l2) and torch.equal(l1, l3), (G, B)
            assert torch.equal(c1, c2), (G, B)
    # the counts of the first draw against the oracle at the parity bar
    _, cq, _ = oracle.forward(spec, draws[0])
    sel = cq >= 1e-6 * cq.max()
    assert np.max(np.abs(c2[0].cpu().numpy()[sel] - cq[sel]) / cq[sel]) < 1e-4


def test_noalloc_size_limit_and_errors(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1()                               # 128x128 cells, 128 phases, 256 energies
    plan = ppm.Plan(spec, max_batch=8)
    dt = torch.zeros((plan.n_phase, plan.n_chan), dtype=torch.int32, device=dev)
    pt = torch.tensor(np.tile(p, (8, 1)), dtype=torch.float64, device=dev)
    l1 = plan.loglike_noalloc(pt[:1].contiguous(), dt)      # one instance fits with one ring per group
    assert torch.equal(l1, plan.loglike(pt[:1].contiguous(), dt))
    with pytest.raises(ppm.PPMError, match="64 MiB"):
        plan.loglike_noalloc(pt[:2].contiguous(), dt)
    plan.set_tiles(ring_group=16)
    l4 = plan.loglike_noalloc(pt[:4].contiguous(), dt)      # four with groups of 16 rings
    assert torch.equal(l4, plan.loglike(pt[:4].contiguous(), dt))
    with pytest.raises(ppm.PPMError, match="64 MiB"):
        plan.loglike_noalloc(pt, dt)
    mspec, mp, mm = syn.map_config(4, "full", n_phase=8, n_energy=16)
    mplan = ppm.Plan(mspec, max_batch=1)
    with pytest.raises(ppm.PPMError, match="map"):
        mplan.loglike_noalloc(torch.tensor(mp[None], dtype=torch.float64, device=dev),
                              torch.zeros((8, mplan.n_chan), dtype=torch.int32, device=dev))
