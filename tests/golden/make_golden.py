"""Writes the stored expected values used by the full-size parity tests.

Calls only the FP64 CPU oracle (and the seeded input generators):
  config1_counts.npy  expected counts [128, 300] of the config-1 workload
                      (oblate star, cap + annulus, 128x128 cells per spot,
                      128 phases, 256 energies, 300 channels)
  config1_data.npy    seeded Poisson draw (seed 13) from those counts, int32
  config1_meta.json   oracle diagnostics and input digests
Run: python tests/golden/make_golden.py   (about a minute on 8 cores)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synthetic as syn  # noqa: E402


def main():
    spec, p = syn.config1()
    ft, cnt, diag = oracle.forward(spec, p)
    data = syn.poisson_data(cnt)
    np.save(os.path.join(HERE, "config1_counts.npy"), cnt)
    np.save(os.path.join(HERE, "config1_data.npy"), data)
    meta = dict(diag=diag, params=p.tolist(),
                digest_atmos=syn.digest(spec["atmos_logI"]), digest_rsp=syn.digest(spec["rsp"]),
                loglike=oracle.loglike_from_counts(cnt, data), flux_max=float(ft.max()))
    with open(os.path.join(HERE, "config1_meta.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(meta)


if __name__ == "__main__":
    main()
