"""Writes stored oracle photon flux before absorption and response (F_t of
Eq. 47, [phase][energy]) for the full-size flux parity tests, and the
counts of one 512x512-cell instance of the uneven-resolution batch.

Calls only the FP64 CPU oracle (and the seeded input generators):
  config1_flux.npy     F_t [128, 256] of the benchmark workload (128x128 cells
                       per spot, 128 phases, 256 energies)
  config2_flux.npy     F_t [256, 256] of the stress workload at full size
                       (512x512 cells per spot, 512 fine phases, 256 phases)
  config3_counts.npz   adds "res512": counts [128, 300] of the first draw
                       (seed 14) whose grid (seed 15) is 512 cells per side,
                       on the cap + annulus spec (its index and diagnostics go
                       to large_meta.json as "config3_res512")
Run: python tests/golden/make_golden_flux.py   (about an hour on 8 cores)
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
    spec, p = syn.config1()
    ft, cnt, diag = oracle.forward(spec, p)
    ref = np.load(os.path.join(HERE, "config1_counts.npy"))
    assert np.allclose(cnt, ref, rtol=1e-12, atol=0), "config-1 counts differ from the stored ones"
    np.save(os.path.join(HERE, "config1_flux.npy"), ft)
    print("config1 flux %.0f s" % (time.time() - t0), flush=True)

    meta_path = os.path.join(HERE, "large_meta.json")
    meta = json.load(open(meta_path))
    draws, res = syn.config3_draws()
    i = int(np.argmax(res == 512))
    spec, _ = syn.config1(n_cells=512)
    _, cnt, diag = oracle.forward(spec, draws[i])
    npz = os.path.join(HERE, "config3_counts.npz")
    old = dict(np.load(npz))
    old["res512"] = cnt
    np.savez(npz, **old)
    meta["config3_res512"] = dict(index=i, diag=diag)
    with open(meta_path, "w") as f:
        json.dump(meta, f, indent=1)
    print("config3 512 draw %d %.0f s" % (i, time.time() - t0), flush=True)

    spec, p = syn.config2()
    ft, cnt, diag = oracle.forward(spec, p)
    ref = np.load(os.path.join(HERE, "config2_counts.npy"))
    assert np.allclose(cnt, ref, rtol=1e-12, atol=0), "config-2 counts differ from the stored ones"
    np.save(os.path.join(HERE, "config2_flux.npy"), ft)
    print("config2 flux %.0f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
