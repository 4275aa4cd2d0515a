"""Writes stored oracle counts of the full-surface temperature-map workload:
n_side 64 (49,152 HEALPix patches, every one active: smooth background with
a hot polar-cap-like region and an arc), the config-1 star, 128 phases, 256
energies, 300 channels, synthetic atmosphere, absorption and response.

Calls only the FP64 CPU oracle (and the seeded input generators):
  map64_counts.npy   counts [128, 300]
  map64_meta.json    oracle diagnostics
Run: python tests/golden/make_golden_map.py   (about a minute on 8 cores)
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
    spec, p, m = syn.map_config(64, "full")
    _, cnt, diag = oracle.forward_map(spec, p, 64, m)
    np.save(os.path.join(HERE, "map64_counts.npy"), cnt)
    with open(os.path.join(HERE, "map64_meta.json"), "w") as f:
        json.dump(dict(diag=diag, digest_map=syn.digest(m), seconds=time.time() - t0), f, indent=1)
    print("map64 %.0f s" % (time.time() - t0), diag, flush=True)


if __name__ == "__main__":
    main()
