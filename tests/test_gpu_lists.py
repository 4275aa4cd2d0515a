"""GPU checks of the plan's resident work lists (``include/ppm.h``, work
lists): uploads are ordered on the caller's stream, so that calls with
changing batch layouts on a non-default stream, with no host
synchronisation in between, give the results of their single calls bit
for bit; a layout used under HIP graph capture is pinned, so that direct
calls with other layouts between replays leave the graph's results
unchanged."""
import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def layouts(n, B, seed=3):
    rng = np.random.default_rng(seed)
    return [np.ascontiguousarray(2 * rng.integers(1, 7, size=B), dtype=np.int32) for _ in range(n)]


def test_changing_layouts_on_a_side_stream(torch_dev):
    """Twelve layouts (more than the plan keeps) cycled twice on a side
    stream with no host sync: every call re-uploads its lists while earlier
    calls' kernels may still be queued."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, _ = syn.config1(n_cells=12, n_phase=16, n_energy=64)
    draws, _ = syn.config3_draws(4)
    B = 4
    plan = ppm.Plan(spec, max_batch=B, max_cells=12)
    pt = torch.tensor(draws[:B], dtype=torch.float64, device=dev)
    lay = layouts(12, B)
    ref = []
    for nc in lay:
        ref.append(plan.forward(pt, n_cells=nc).cpu().numpy())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    outs = []
    with torch.cuda.stream(side):
        for rep in range(2):
            for nc in lay:
                outs.append(plan.forward(pt, n_cells=nc))
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), ref[i % len(lay)]), i
    # the same with a ring-group size (lists of groups change with it)
    plan.set_tiles(ring_group=3)
    ref3 = [plan.forward(pt, n_cells=nc).cpu().numpy() for nc in lay[:3]]
    with torch.cuda.stream(side):
        outs = [plan.forward(pt, n_cells=lay[i % 3]) for i in range(9)]
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), ref3[i % 3]), i


def test_graph_survives_direct_calls_with_other_layouts(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=12, n_phase=16, n_energy=64)
    from oracle import forward
    _, cnt, _ = forward(spec, p)
    dt = torch.tensor(syn.poisson_data(cnt), device=dev)
    draws, _ = syn.config3_draws(3)
    B = 3
    plan = ppm.Plan(spec, max_batch=B, max_cells=12)
    pt = torch.tensor(draws[:B], dtype=torch.float64, device=dev)
    lay = layouts(11, B, seed=5)
    gl = ppm.GraphedLogLike(plan, dt, B, n_cells=lay[0])
    want = plan.loglike(pt, dt, n_cells=lay[0]).clone()
    for rep in range(3):
        for nc in lay[1:]:                       # evict every unpinned slot, several times
            plan.loglike(pt, dt, n_cells=nc)
        got = gl(pt).clone()
        torch.cuda.synchronize()
        assert torch.equal(got, want), rep
    # a second graph of another layout on the same plan keeps its own lists
    gl2 = ppm.GraphedLogLike(plan, dt, B, n_cells=lay[1])
    want2 = plan.loglike(pt, dt, n_cells=lay[1]).clone()
    plan.loglike(pt, dt, n_cells=lay[2])
    assert torch.equal(gl(pt).clone(), want) and torch.equal(gl2(pt).clone(), want2)


def test_capture_needs_a_resident_layout_and_slots_run_out(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=8, n_phase=8, n_energy=32)
    draws, _ = syn.config3_draws(2)
    plan = ppm.Plan(spec, max_batch=2, max_cells=8)
    pt = torch.tensor(draws[:2], dtype=torch.float64, device=dev)
    out = torch.empty((2, plan.n_phase, plan.n_chan), dtype=torch.float64, device=dev)
    nc_new = np.array([2, 4], dtype=np.int32)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with pytest.raises(ppm.PPMError, match="resident"):
        with torch.cuda.graph(g, stream=side):
            plan.forward(pt, n_cells=nc_new, out=out)
    torch.cuda.synchronize()
    ref = plan.forward(pt, n_cells=nc_new).cpu().numpy()
    # eight captured layouts pin every slot: a ninth layout is refused, the
    # pinned ones keep working
    dt = torch.zeros((plan.n_phase, plan.n_chan), dtype=torch.int32, device=dev)
    lay = [np.array([2 * (i % 4 + 1), 2 * (i // 4 + 1)], dtype=np.int32) for i in range(9)]
    graphs = [ppm.GraphedLogLike(plan, dt, 2, n_cells=lay[i]) for i in range(8)]
    with pytest.raises(ppm.PPMError, match="captured graph"):
        plan.forward(pt, n_cells=lay[8])
    got = plan.forward(pt, n_cells=lay[3]).cpu().numpy()
    assert np.all(np.isfinite(got))
    for gr in graphs:
        assert torch.all(torch.isfinite(gr(pt)))
    assert ref.shape == (2, plan.n_phase, plan.n_chan)
