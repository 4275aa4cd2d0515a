"""Writes the oracle's stress workload at twice the surface resolution
(1024x1024 cells per spot, everything else as at full size: 512 fine
phases, 256 phases, 256 energies, 300 channels), the reference for the
discretisation error of the 512x512 grid (the resolution tiers of Sect. 5).
It is reported, not gated: the GPU at 512x512 against this reference
measures the surface discretisation, not the implementation.

Calls only the FP64 CPU oracle (and the seeded input generators):
  config2_1024_counts.npy  counts [256, 300]
  config2_1024_flux.npy    F_t [256, 256] before absorption and response
  config2_1024_meta.json   oracle diagnostics and run time
Run: python tests/golden/make_golden_res.py   (several hours on 8 cores)
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
    spec, p = syn.config2(n_cells=1024)
    ft, cnt, diag = oracle.forward(spec, p)
    np.save(os.path.join(HERE, "config2_1024_counts.npy"), cnt)
    np.save(os.path.join(HERE, "config2_1024_flux.npy"), ft)
    with open(os.path.join(HERE, "config2_1024_meta.json"), "w") as f:
        json.dump(dict(diag=diag, seconds=time.time() - t0, cells=1024), f, indent=1)
    print("config2 at 1024 cells %.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
