"""Benchmark: forward + Poisson log-likelihood evaluations per second on the
config-1 workload (oblate 600 Hz star, a circular cap and an annulus,
128x128 cells per spot, 128 phases, 256 energies, 300 channels, synthetic
atmosphere table, absorption and response), on one MI355X.

A step is one full evaluation of the hot path (setup, FP64 deflection
tables, fine-phase traces, atmosphere collapse, intensity accumulation,
ring reduction and absorption, MFMA response fold, FP64 log-likelihood) for
one parameter vector, inputs resident in device memory.

Prints one JSON line.  `value` is the plain (one vector per call) rate; the
graph-replayed plain rate, the batched rates (B vectors per call), the
uneven-resolution sampler batch (1024 draws with their own grids) and the
+grad rate (logL and its twelve-parameter gradient, B vectors per call) are
reported beside it.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "forward+logL evals/sec at config[1], plain vs batched vs +grad, <=1e-4 rel err"
# Algorithmic FP32 work per (cell, phase, energy) unit of the intensity
# accumulation: x index and fraction 3, cubic Lagrange weights 10, 4-term
# dot 7, scale and accumulate 2; plus the mu contraction of the ~63 x nodes
# an energy window touches (8 FLOP each) amortised over 256 energies (~2).
FLOP_PER_UNIT = 24.0
# Temperature-map accumulation: the same per-energy work plus the second
# logT slab in the mu contraction (8 FLOP) and the logT blend (2 FLOP) at
# each of the ~63 x nodes of a pair, amortised over 256 energies (~2.5).
FLOP_PER_UNIT_MAP = 26.5
PEAK_FP32_TFLOPS = 157.3

# HBM traffic of the hot kernel per launch (config-1 workload, one vector),
# per phase tile of the launch: FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
# from rocprofv3 --pmc runs, one counter per run, each scaled by what the same
# counter reads for a 256 MiB device-to-device copy (FETCH_SIZE reads half the
# copied bytes on this part, WRITE_SIZE all of them).  Valid only for the
# kernel sources the counters were taken on and for the tiles listed; any
# other case reports null until the counters are taken again.
KERNEL_SOURCES = ("ppm_kernels.hip", "ppm_device.h", "ppm_dual.h", "ppm_internal.h", "ppm_launch.h")
TRAFFIC = {"sources_sha256": "fdd32e6f6973e23cf971741f6ced43d21969141b1c91166e28389d80d68cbd4f",
           "fetch_scale": 1.99980, "write_scale": 1.0,
           # phase tile -> (FETCH_SIZE, WRITE_SIZE) KiB per dispatch
           "by_tile": {64: (4316.63, 32960.00), 128: (4316.56, 32864.00)},
           "profile": "profiles/k_accum_fast_config1_traffic.md"}


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_07764_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hot_kernel_traffic(phase_tile):
    """HBM bytes per launch of the hot kernel, or None when the counters were
    taken on other kernel sources or another launch shape."""
    t = TRAFFIC
    if t["sources_sha256"] is None or t["sources_sha256"] != kernel_sources_sha256():
        return None
    if phase_tile not in t["by_tile"]:
        return None
    fetch_kib, write_kib = t["by_tile"][phase_tile]
    return (fetch_kib * t["fetch_scale"] + write_kib * t["write_scale"]) * 1024.0


def cpu_baseline(sample_cells: int, one_core_cells: int):
    """The FP64 oracle timed on the host: all cores (at most 16, the box's
    share) on sample_cells per spot, and one core on one_core_cells per spot;
    work is linear in the number of cells, so each is scaled to the whole
    workload."""
    import oracle
    import synthetic as syn

    def run(cells, threads):
        oracle.set_threads(threads)
        spec, p = syn.config1(n_cells=cells)
        os_ = oracle.OracleSpec(spec)
        t0 = time.perf_counter()
        _, cnt, _ = oracle.forward(os_, p)
        data = syn.poisson_data(cnt)
        oracle.loglike_from_counts(cnt, data)
        dt = time.perf_counter() - t0
        scale = (128.0 / cells) ** 2
        return dt, scale

    threads = min(os.cpu_count() or 1, 16)
    dt, scale = run(sample_cells, threads)
    out = {"value": 1.0 / (dt * scale), "unit": "evals/s", "cores": threads, "kind": "oracle",
           "sample": f"config-1 workload at {sample_cells}x{sample_cells} cells per spot "
                     f"({'the whole workload' if scale == 1 else f'1/{scale:.0f} of the cells, scaled linearly'}; "
                     f"all phases/energies/channels), {dt:.2f} s on {threads} threads"}
    if one_core_cells > 0:
        dt1, scale1 = run(one_core_cells, 1)
        out["one_core"] = {"value": 1.0 / (dt1 * scale1), "unit": "evals/s", "cores": 1,
                           "sample": f"{one_core_cells}x{one_core_cells} cells per spot (1/{scale1:.0f} of the "
                                     f"cells), {dt1:.2f} s, scaled linearly"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=256, help="vectors per call in the batched leg (0: skip)")
    ap.add_argument("--batch-large", type=int, default=1024,
                    help="vectors per call in the second batched leg (0: skip)")
    ap.add_argument("--grad-batch", type=int, default=256, help="vectors per call in the +grad leg (0: skip)")
    ap.add_argument("--cpu-one-core", type=int, default=32,
                    help="cells per spot of the single-core oracle sample (0: skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run device-to-device copies of this many MiB (HBM counter calibration; 0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=128,
                    help="cells per spot of the oracle sample (128: the whole workload; 0: skip)")
    ap.add_argument("--map-nside", type=int, default=64,
                    help="HEALPix n_side of the full-surface temperature-map leg (0: skip)")
    ap.add_argument("--map-batch", type=int, default=32, help="vectors per call in the batched map leg (0: skip)")
    ap.add_argument("--map-tile", default="auto", help="phase tile of the map legs: 'auto' or 8, 16, 32")
    ap.add_argument("--pt-chains", type=int, default=64, help="chains per temperature of the sampler leg (0: skip)")
    ap.add_argument("--pt-temps", type=int, default=4, help="temperatures of the sampler leg")
    ap.add_argument("--pt-steps", type=int, default=20, help="timed steps of the sampler leg")
    ap.add_argument("--tiles", default="auto",
                    help="launch shape of the accumulation kernels: 'auto' (autotuner, per leg) or "
                         "'F,G[,R]' (forward and adjoint phase tiles, rings per forward work-group)")
    ap.add_argument("--uneven", type=int, default=1024,
                    help="seeded sampler draws with their own grids (64..512 cells per side) per call of the "
                         "uneven-resolution leg (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the batched path shards "
              "parameter vectors across GPUs by design, but this program measures one GPU",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2510_07764_amd as ppm
    import synthetic as syn

    dev = torch.device("cuda:0")
    spec, p = syn.config1()
    gold = os.path.join(ROOT, "tests", "golden", "config1_data.npy")
    data = np.load(gold)
    data_t = torch.tensor(data, device=dev)

    def tune(plan_, params_, reps, n_cells=None):
        """Autotuned (or fixed) launch shape of a plan; returns the report."""
        if args.tiles == "auto":
            rep = plan_.autotune(params_, n_cells=n_cells, reps=reps)
            return {"chosen": list(rep["chosen"]), "ring_group": rep["ring_group"],
                    "forward_ms": {str(k): round(v, 4) for k, v in rep["forward"].items()},
                    "group_ms": {str(k): round(v, 4) for k, v in rep["group"].items()},
                    "grad_ms": {str(k): round(v, 4) for k, v in rep["grad"].items()}}
        f, g, r = (int(v) for v in (args.tiles.split(",") + ["1"])[:3])
        plan_.set_tiles(f, g, r)
        return {"chosen": [f, g], "ring_group": r, "fixed": True}

    def prewarm(fn, seconds=0.2):
        """Untimed calls for about `seconds` (the GPU clock ramps up under
        sustained load and drops when idle), before a leg's warm-up calls."""
        t_end = time.perf_counter() + seconds
        n = 0
        while time.perf_counter() < t_end:
            fn()
            n += 1
            if n % 16 == 0:
                torch.cuda.synchronize()
        torch.cuda.synchronize()

    # ---------------- plain: one parameter vector per call
    plan = ppm.Plan(spec, max_batch=1)
    pt = torch.tensor(p[None], dtype=torch.float64, device=dev)
    tune_plain = tune(plan, pt, 10)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    prewarm(lambda: plan.loglike(pt, data_t, out=ll))
    for _ in range(args.warmup):
        plan.loglike(pt, data_t, out=ll)
    # the hot kernel is timed with HIP events on the last fifth of the timed
    # calls: each event pair adds a few microseconds of stream work, which
    # would otherwise be charged to every call (events created here, outside)
    n_prof = max(1, args.steps // 5)
    plan.profile_begin(n_prof)
    plan.profile_end()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - n_prof:
            plan.profile_begin(n_prof)
        plan.loglike(pt, data_t, out=ll)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hot_ms, n_hot = plan.profile_end()
    plain_s = (t1 - t0) / args.steps
    pairs = plan.visible_pairs(1)
    units = pairs * plan.n_energy
    hot_avg_s = hot_ms / max(n_hot, 1) * 1e-3
    achieved = units * FLOP_PER_UNIT / hot_avg_s / 1e12

    # ---------------- plain, graph-replayed: the same single-vector call
    # submitted as one captured HIP graph per evaluation
    gl1 = ppm.GraphedLogLike(plan, data_t, 1)
    prewarm(lambda: gl1(pt))
    for _ in range(args.warmup):
        gl1(pt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gl1(pt)
    torch.cuda.synchronize()
    plain_graph_s = (time.perf_counter() - t0) / args.steps
    graph_ok = bool(torch.equal(gl1(pt), ll))
    del gl1

    # ---------------- batched: B vectors per graph replay; config-1-shape draws,
    # or the uneven-resolution sampler draws with their own grids
    def batched_leg(B, uneven=False, tiles_from=None):
        if uneven:
            draws, res = syn.config3_draws(B)
            nc = np.ascontiguousarray(res, dtype=np.int32)
            planb = ppm.Plan(spec, max_batch=B, max_cells=int(nc.max()))
        else:
            draws, nc = syn.config4_draws(B), None
            planb = ppm.Plan(spec, max_batch=B)
        ptb = torch.tensor(draws, dtype=torch.float64, device=dev)
        if tiles_from is None:
            tuned = tune(planb, ptb, 3, n_cells=nc)
        else:
            # one evaluation of this leg takes seconds: the launch shape tuned on
            # the large config-1-shape batch is taken over instead of re-tuned
            f, g = tiles_from["chosen"]
            planb.set_tiles(f, g, tiles_from["ring_group"])
            tuned = {"chosen": [f, g], "ring_group": tiles_from["ring_group"], "from": "batched_large"}
        prewarm(lambda: planb.loglike(ptb, data_t, n_cells=nc))
        # one direct call with the hot kernel timed (events on the launch stream)
        planb.profile_begin(64)
        planb.loglike(ptb, data_t, n_cells=nc)
        torch.cuda.synchronize()
        hms, nh = planb.profile_end()
        bunits = planb.visible_pairs(B) * planb.n_energy
        passes = planb.passes
        glb = ppm.GraphedLogLike(planb, data_t, B, n_cells=nc)
        glb(ptb)
        torch.cuda.synchronize()
        kb = max(5, args.steps // 10)
        t0 = time.perf_counter()
        for _ in range(kb):
            out_b = glb(ptb)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / kb
        bach = bunits * FLOP_PER_UNIT / (hms * 1e-3) / 1e12
        out = {"evals_per_s": B / tb, "batch": B, "ms_per_call": tb * 1e3, "calls": kb, "passes": passes,
               "finite": bool(torch.isfinite(out_b).all().item()),
               "n_finite": int(torch.isfinite(out_b).sum().item()), "vs_plain": (B / tb) * plain_s,
               "hot_kernel_ms": hms, "hot_kernel_launches": nh, "units": bunits,
               "roofline_frac": bach / PEAK_FP32_TFLOPS, "tiles": tuned}
        if uneven:
            out["grids"] = {str(n): int((nc == n).sum()) for n in (64, 128, 256, 512)}
            out["workload"] = (f"{B} seeded sampler draws (M 1-2.2, R_e 9-15 km, any geometry, logT 5.8-6.6) with "
                               f"per-instance grids 64^2..512^2 cells per spot, 128 phases, 256 energies, "
                               f"300 channels; one captured graph per call; logL is -inf where a "
                               f"draw's spots leave a phase bin dark (model counts 0 where the data "
                               f"count is positive)")
        del glb, planb
        return out

    batched = batched_leg(args.batch) if args.batch > 0 else None
    batched_large = batched_leg(args.batch_large) if args.batch_large > 0 else None
    uneven = None
    if args.uneven > 0:
        uneven = batched_leg(args.uneven, uneven=True,
                             tiles_from=batched_large["tiles"] if batched_large is not None else None)

    # ---------------- +grad: logL and the twelve-parameter gradient, B vectors per graph replay
    grad = None
    if args.grad_batch > 0:
        B = args.grad_batch
        draws = syn.config4_draws(B)
        plang = ppm.Plan(spec, max_batch=B, grad=True)
        ptg = torch.tensor(draws, dtype=torch.float64, device=dev)
        tuned_g = tune(plang, ptg, 2)
        glg = ppm.GraphedLogLike(plang, data_t, B, grad=True)
        prewarm(lambda: glg(ptg))
        kg = max(5, args.steps // 10)
        t0 = time.perf_counter()
        for _ in range(kg):
            out_l, out_g = glg(ptg)
        torch.cuda.synchronize()
        tg = (time.perf_counter() - t0) / kg
        grad = {"evals_per_s": B / tg, "batch": B, "ms_per_call": tg * 1e3, "calls": kg,
                "finite": bool(torch.isfinite(out_g).all().item()),
                "vs_plain": (B / tg) * plain_s, "tiles": tuned_g}
        del glg, plang

    # ---------------- GPU-resident parallel-tempered sampler on workload 1: every
    # step one batched likelihood call of chains x temperatures proposals
    ptleg = None
    if args.pt_chains > 0:
        Cc, Tt = args.pt_chains, args.pt_temps
        betas = [0.5 ** t for t in range(Tt)]
        free = list(syn.GRAD_SLOTS)
        lo = [p[s] * 0.9 if p[s] > 0 else -0.5 for s in free]
        hi = [p[s] * 1.1 if p[s] > 0 else 0.5 for s in free]
        steps = [max(abs(p[s]), 0.05) * 2e-3 for s in free]
        pplan = ppm.Plan(spec, max_batch=Cc * Tt)
        ptune = tune(pplan, torch.tensor(syn.config4_draws(Cc * Tt), dtype=torch.float64, device=dev), 2)
        sampler = ppm.PTSampler(Cc, betas, free, lo, hi, steps, seed=2025, swap_every=1)
        start = torch.tensor(np.tile(p, (Tt, Cc, 1)), dtype=torch.float64, device=dev)
        sampler.set_state(start)
        sampler.run(pplan, data_t, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, chain_l = sampler.run(pplan, data_t, args.pt_steps)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) / args.pt_steps
        _, _, nacc, nsw, _ = sampler.state()
        ptleg = {"chains": Cc, "temperatures": Tt, "steps": args.pt_steps, "ms_per_step": tp * 1e3,
                 "steps_per_s": 1.0 / tp, "loglike_evals_per_s": Cc * Tt / tp,
                 "accept_rate": float(nacc.sum().item()) / ((args.pt_steps + 2) * Cc * Tt),
                 "swap_rate": (float(nsw.sum().item()) / ((args.pt_steps + 2) * Cc * max(Tt - 1, 1) / 2)
                               if Tt > 1 else None),
                 "finite": bool(torch.isfinite(chain_l).all().item()), "tiles": ptune}
        del sampler, pplan

    # ---------------- full-surface temperature map (HEALPix), one vector per call,
    # then a batch of maps (the same map, parameter draws of the batched leg)
    tmap = None
    if args.map_nside > 0:
        mspec, mp, mm = syn.map_config(args.map_nside, "full")
        mplan = ppm.Plan(mspec, max_batch=max(1, args.map_batch))
        mpt = torch.tensor(mp[None], dtype=torch.float64, device=dev)
        mmt = torch.tensor(mm[None], dtype=torch.float64, device=dev)
        mll = torch.empty(1, dtype=torch.float64, device=dev)
        mtune = None
        if args.map_tile == "auto":
            r = mplan.autotune_map(mpt, mmt, reps=5)
            mtune = {"chosen": r["chosen"][0], "forward_ms": {str(k): round(v, 4) for k, v in r["forward"].items()}}
        else:
            mplan.set_tiles(phase_tile=int(args.map_tile))
            mtune = {"chosen": int(args.map_tile), "fixed": True}
        prewarm(lambda: mplan.loglike_map(mpt, mmt, data_t, out=mll))
        for _ in range(args.warmup):
            mplan.loglike_map(mpt, mmt, data_t, out=mll)
        mplan.profile_begin(n_prof)          # events on the last fifth, as in the plain leg
        mplan.profile_end()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            if i == args.steps - n_prof:
                mplan.profile_begin(n_prof)
            mplan.loglike_map(mpt, mmt, data_t, out=mll)
        torch.cuda.synchronize()
        map_s = (time.perf_counter() - t0) / args.steps
        mhot, mn = mplan.profile_end()
        munits = mplan.visible_pairs(1) * mplan.n_energy
        mhot_s = mhot / max(mn, 1) * 1e-3
        mach = munits * FLOP_PER_UNIT_MAP / mhot_s / 1e12
        tmap = {"workload": f"full-surface map, HEALPix n_side {args.map_nside} "
                            f"({12 * args.map_nside ** 2} patches, all active), config-1 star and instrument",
                "evals_per_s": 1.0 / map_s, "ms_per_call": map_s * 1e3,
                "kernel": "k_accum_map", "kernel_ms": mhot_s * 1e3, "units": munits,
                "flop_per_unit": FLOP_PER_UNIT_MAP, "achieved": mach, "frac": mach / PEAK_FP32_TFLOPS,
                "logL": float(mll.item()), "tiles": mtune}
        if args.map_batch > 1:
            Bm = args.map_batch
            mptb = torch.tensor(np.tile(mp, (Bm, 1)), dtype=torch.float64, device=dev)
            mptb[:, 3] = torch.linspace(0.0, 0.5, Bm, dtype=torch.float64)
            mmtb = mmt.repeat(Bm, 1).contiguous()
            mllb = torch.empty(Bm, dtype=torch.float64, device=dev)
            mtune_b = {"chosen": mplan.tiles[0], "fixed": True}
            if args.map_tile == "auto":
                r = mplan.autotune_map(mptb, mmtb, reps=2)
                mtune_b = {"chosen": r["chosen"][0],
                           "forward_ms": {str(k): round(v, 4) for k, v in r["forward"].items()}}
            mplan.loglike_map(mptb, mmtb, data_t, out=mllb)
            torch.cuda.synchronize()
            kmb = max(2, args.steps // 10)
            t0 = time.perf_counter()
            for _ in range(kmb):
                mplan.loglike_map(mptb, mmtb, data_t, out=mllb)
            torch.cuda.synchronize()
            tmb = (time.perf_counter() - t0) / kmb
            tmap["batched"] = {"batch": Bm, "evals_per_s": Bm / tmb, "ms_per_call": tmb * 1e3,
                               "finite": bool(torch.isfinite(mllb).all().item()), "tiles": mtune_b}
        del mplan

    if args.copy_mib > 0:
        # plain copy kernel of known size: reads and writes copy_mib MiB each
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = cpu_baseline(args.cpu_sample, args.cpu_one_core) if args.cpu_sample > 0 else None
    out = {
        "metric": METRIC,
        "value": 1.0 / plain_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": plain_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "config-1: oblate 600 Hz star, cap + annulus, 128x128 cells per spot, "
                               "128 phases, 256 energies, 300 channels, synthetic atmosphere, absorption, response",
                   "plain": "one parameter vector per call", "logL": float(ll.item())},
        "plain_graph": {"evals_per_s": 1.0 / plain_graph_s, "ms_per_call": plain_graph_s * 1e3,
                        "matches_direct": graph_ok},
        "plain_tiles": tune_plain,
        "batched": batched,
        "batched_large": batched_large,
        "uneven": uneven,
        "grad": grad,
        "map": tmap,
        "sampler": ptleg,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": hot_kernel_traffic(plan.tiles[0]),
                     "kernel": "k_accum_fast<4, 12>", "kernel_ms": hot_avg_s * 1e3, "units": units,
                     "flop_per_unit": FLOP_PER_UNIT},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
