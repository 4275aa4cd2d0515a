"""Writes stored oracle counts for the full-size parity tests of the stress
workload and of sampled instances of the uneven-resolution batch.

Calls only the FP64 CPU oracle (and the seeded input generators):
  config2_counts.npy   counts [256, 300] of the stress workload at full size:
                       compactness 0.28, pole-straddling cap (1.2 rad) and a
                       near-grazing crescent, 512x512 cells per spot, 512
                       fine phases, 256 phases, 256 energies
  config3_counts.npz   counts [128, 300] of the first draws (seed 14) whose
                       per-instance grids (seed 15) are 64, 128 and 256
                       cells per side, on the cap + annulus spec
  large_meta.json      draw indices, resolutions and oracle diagnostics
Run: python tests/golden/make_golden_large.py   (about an hour on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synthetic as syn  # noqa: E402


def main():
    t0 = time.time()
    meta = {}
    draws, res = syn.config3_draws()
    picks = {}
    for i, n in enumerate(res):
        if int(n) in (64, 128, 256) and int(n) not in picks:
            picks[int(n)] = i
    out = {}
    for n, i in sorted(picks.items()):
        spec, _ = syn.config1(n_cells=n)
        _, cnt, diag = oracle.forward(spec, draws[i])
        out["res%d" % n] = cnt
        meta["config3_res%d" % n] = dict(index=i, diag=diag)
        print("config3", n, i, "%.0f s" % (time.time() - t0), flush=True)
    np.savez(os.path.join(HERE, "config3_counts.npz"), **out)
    spec, p = syn.config2()
    _, cnt, diag = oracle.forward(spec, p)
    np.save(os.path.join(HERE, "config2_counts.npy"), cnt)
    meta["config2"] = dict(diag=diag)
    print("config2 %.0f s" % (time.time() - t0), flush=True)
    with open(os.path.join(HERE, "large_meta.json"), "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
