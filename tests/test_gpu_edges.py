"""GPU parity of the less travelled paths and of degenerate inputs, through
the C ABI, against the FP64 oracle (bar: 1e-4 relative per bin at or above
1e-6 of the peak, as for the main workload).

* an energy grid wider than the windowed kernel's 59 x intervals (0.1-10
  keV): the generic accumulation kernel, with energies leaving the
  atmosphere table's x axis (zero contribution there);
* 400 energies (8 per lane in the windowed kernel);
* the spherical (S+D) star with the atmosphere table;
* pole-on observer (a flat light curve), a spot centred on the pole, a
  single cell per spot with one phase and one energy;
* argument errors of the evaluation calls;
* coarse fine-phase traces on a fast spinner, where the redshift changes by
  more than 1/16 between fine samples (the windowed kernel's x positions
  then take their halving path, and phase buckets hold several samples).
"""
import math

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


def run(torch_dev, spec, params, **kw):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    p = np.atleast_2d(params)
    plan = ppm.Plan(spec, max_batch=p.shape[0], **kw)
    out = plan.forward(torch.tensor(p, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    return out.cpu().numpy(), plan


def with_energy(spec, energy):
    s = dict(spec, energy=energy)
    syn.attach_instrument(s)
    return s


def test_wide_energy_grid_generic_kernel(torch_dev):
    import paper_2510_07764_amd as ppm
    spec, p = syn.config1(n_cells=12, n_phase=16, n_energy=48)
    spec = with_energy(spec, syn.logspace(0.1, 10.0, 48))
    _, cnt, diag = oracle.forward(spec, p)
    got, _ = run(torch_dev, spec, p)
    err = rel_err(got[0], cnt)
    print("wide grid: err %.2e, x outside the table: %d" % (err, diag["n_x_outside"]))
    assert diag["n_x_outside"] > 0
    assert err < TOL
    with pytest.raises(ppm.PPMError, match="59"):
        ppm.Plan(spec, max_batch=1, grad=True)


def test_many_energies(torch_dev):
    spec, p = syn.config1(n_cells=10, n_phase=12, n_energy=400)
    _, cnt, _ = oracle.forward(spec, p)
    got, _ = run(torch_dev, spec, p)
    err = rel_err(got[0], cnt)
    print("400 energies: err %.2e" % err)
    assert err < TOL


def test_spherical_star_with_table(torch_dev):
    spec, p = syn.config1(n_cells=12, n_phase=20, n_energy=40)
    spec = dict(spec, mode=syn.MODE_SD)
    _, cnt, _ = oracle.forward(spec, p)
    got, _ = run(torch_dev, spec, p)
    err = rel_err(got[0], cnt)
    print("S+D with table: err %.2e" % err)
    assert err < TOL


def test_pole_on_and_polar_spot(torch_dev):
    spec, p = syn.config1(n_cells=10, n_phase=16, n_energy=32)
    q = p.copy()
    q[2] = 0.0            # observer on the rotation axis: nothing varies with phase
    q[8] = 0.0            # spot 1 centred on the pole
    _, cnt, _ = oracle.forward(spec, q)
    got, _ = run(torch_dev, spec, q)
    err = rel_err(got[0], cnt)
    flat = np.abs(got[0] - got[0].mean(axis=0)).max() / got[0].max()
    print("pole-on: err %.2e, phase variation %.1e" % (err, flat))
    assert err < TOL
    assert flat < 1e-6


def test_single_cell_phase_energy(torch_dev):
    spec, p = syn.config1(n_cells=2, n_phase=1, n_energy=8)
    energy = np.array([1.0])
    spec = dict(spec, n_rings=[1, 2], n_phi=[1, 2], energy=energy, sigma=syn.sigma_ism(energy),
                rsp=np.array([[1.0, 2.0, 0.5]]))
    _, cnt, _ = oracle.forward(spec, p)
    got, _ = run(torch_dev, spec, p)
    assert got.shape == (1, 1, 3)
    err = rel_err(got[0], cnt)
    print("1 phase, 1 energy, 1-cell cap: err %.2e" % err)
    assert err < TOL


def test_call_errors(torch_dev):
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=8, n_phase=8, n_energy=16)
    plan = ppm.Plan(spec, max_batch=2, max_cells=12)
    pt = torch.tensor(np.stack([p, p, p]), dtype=torch.float64, device=dev)
    with pytest.raises(ppm.PPMError, match="batch"):
        plan.forward(pt)                                   # B > max_batch
    with pytest.raises(ppm.PPMError, match="max_cells"):
        plan.forward(pt[:1].contiguous(), n_cells=[16])    # grid beyond max_cells
    with pytest.raises(ppm.PPMError, match="even"):
        plan.forward(pt[:1].contiguous(), n_cells=[9])     # annulus needs an even grid
    with pytest.raises(ppm.PPMError, match="batch|null"):
        plan.forward(pt[:0].contiguous())                  # B = 0 (an empty tensor has no storage)
    # the plan still works after rejected calls
    _, cnt, _ = oracle.forward(spec, p)
    got = plan.forward(pt[:1].contiguous()).cpu().numpy()
    assert rel_err(got[0], cnt) < TOL


@pytest.mark.parametrize("interp", [0, 1, 2, 3])
def test_interpolation_strategies(torch_dev, interp):
    """The four atmosphere interpolation strategies of Sect. 4 (d, a, b, c)
    against the oracle's implementation of the same strategy."""
    spec, p = syn.config1(n_cells=12, n_phase=16, n_energy=40)
    spec = dict(spec, interp=interp)
    _, cnt, _ = oracle.forward(spec, p)
    got, _ = run(torch_dev, spec, p)
    err = rel_err(got[0], cnt)
    print("strategy %d: err %.2e" % (interp, err))
    assert err < TOL


@pytest.mark.parametrize("test", [1, 2])
def test_interpolation_test_geometries(torch_dev, test):
    """The interpolation-test geometries of Sect. 4 on the steep-limb
    synthetic table: flux before absorption and response, per strategy,
    against the oracle."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.interp_test_geometry(test)
    for mode in (0, 1, 2, 3):
        s = dict(spec, interp=mode)
        ft, _, _ = oracle.forward(s, p)
        plan = ppm.Plan(s, max_batch=1)
        got = plan.flux(torch.tensor(p[None], dtype=torch.float64, device=dev)).cpu().numpy()[0]
        err = rel_err(got, ft)
        print("test %d strategy %d: err %.2e, min/max %.2e" % (test, mode, err, got.min() / got.max()))
        assert err < TOL


def test_wide_grid_many_energies(torch_dev):
    """Generic kernel with 8 energies per lane (300 energies over 0.1-10 keV)."""
    spec, p = syn.config1(n_cells=8, n_phase=8, n_energy=300)
    spec = with_energy(spec, syn.logspace(0.1, 10.0, 300))
    _, cnt, _ = oracle.forward(spec, p)
    got, _ = run(torch_dev, spec, p)
    err = rel_err(got[0], cnt)
    print("wide grid, 300 energies: err %.2e" % err)
    assert err < TOL


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_blackbody_many_energies(torch_dev, precision):
    """Blackbody model with 200 energies (4 per lane): the FP64 fold, and
    the FP32 fold on the matrix cores."""
    spec, p = syn.config0()
    E = 200
    energy = syn.logspace(0.2, 3.0, E)
    spec = dict(spec, energy=energy, sigma=np.zeros(E), rsp=np.eye(E)[:, ::2].copy(), precision=precision)
    ft, cnt, _ = oracle.forward(spec, p)
    got, _ = run(torch_dev, spec, p)
    err = rel_err(got[0], cnt)
    print("blackbody %s, 200 energies: err %.2e" % (precision, err))
    assert err < (1e-9 if precision == "f64" else TOL)


def test_grad_per_instance_grids(torch_dev):
    """Gradient with per-instance spot grids equals the gradient of plans
    built for those grids."""
    import paper_2510_07764_amd as ppm
    torch, dev = torch_dev
    spec, p = syn.config1(n_cells=8, n_phase=16, n_energy=32)
    _, cnt, _ = oracle.forward(spec, p)
    dt = torch.tensor(syn.poisson_data(cnt), device=dev)
    draws = syn.config4_draws(2)
    pt = torch.tensor(draws, dtype=torch.float64, device=dev)
    plan = ppm.Plan(spec, max_batch=2, max_cells=12, grad=True)
    ll, g = plan.loglike_grad(pt, dt, n_cells=[12, 8])
    for i, n in enumerate((12, 8)):
        s, _ = syn.config1(n_cells=n, n_phase=16, n_energy=32)
        pl = ppm.Plan(s, max_batch=1, grad=True)
        l1, g1 = pl.loglike_grad(pt[i:i + 1].contiguous(), dt)
        np.testing.assert_allclose(g[i].cpu().numpy(), g1[0].cpu().numpy(), rtol=1e-6, atol=1e-9 * g1.abs().max().item())
        assert abs(ll[i].item() - l1[0].item()) <= 1e-9 * abs(l1[0].item())


def _max_z_step(spec, params):
    """Largest relative redshift step between fine samples with flux (oracle)."""
    os_ = oracle.OracleSpec(spec)
    qm = 0.0
    for spot in (0, 1):
        for g in oracle.rings(os_, params, spot):
            tr = oracle.trace_ring(os_, params, g)
            if not tr["visible"]:
                continue
            z, F = np.asarray(tr["z"]), np.asarray(tr["F"])
            lit = (F[:-1] != 0) | (F[1:] != 0)
            step = np.abs(z[1:] / z[:-1] - 1.0)[lit]
            if step.size:
                qm = max(qm, float(step.max()))
    return qm


@pytest.mark.parametrize("n_fp,nu", [(8, 600.0), (12, 716.0)])
def test_coarse_trace_fast_spin(torch_dev, n_fp, nu):
    spec, p = syn.config1(n_cells=16, n_phase=32, n_energy=64)
    spec = dict(spec, n_fp=n_fp)
    p = p.copy()
    p[5] = nu
    assert _max_z_step(spec, p) > 1.0 / 16.0      # the halving path is reached
    _, cnt, _ = oracle.forward(oracle.OracleSpec(spec), p)
    got, _ = run(torch_dev, spec, p)
    err = rel_err(got[0], cnt)
    print(f"n_fp {n_fp}, {nu} Hz: max rel err {err:.3e}", flush=True)
    assert err < TOL
