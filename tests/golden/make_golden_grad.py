"""Writes the stored FP64 finite-difference gradient used by the full-size
gradient parity test.

Calls only the FP64 CPU oracle (and the seeded input generators):
  config4_grad.json  at theta_eval = the first seeded draw (seed 16) within
                     +-5% of the config-1 truth, on the config-1 workload
                     (128x128 cells per spot, 128 phases, 256 energies) and
                     the stored config-1 data: the oracle's logL and its
                     central finite differences over the twelve
                     differentiable slots with steps h_i = s |theta_i| for
                     s in 1e-4, 1e-5, 1e-6, 1e-7 ("fd_<s>"), and the
                     chain-rule differences of the counts contracted with
                     d logL / d m (oracle.fd_gradient_counts) for s in
                     1e-5, 3e-6, 1e-6, 3e-7, 1e-7 ("fdc_<s>").
Steps already present in an existing file are kept (each step set takes
about 20 minutes on 8 cores).
Run: python tests/golden/make_golden_grad.py
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

STEPS = (1e-4, 1e-5, 1e-6, 1e-7)
CHAIN_STEPS = (1e-5, 3e-6, 1e-6, 3e-7, 1e-7)


def main():
    path = os.path.join(HERE, "config4_grad.json")
    spec, _ = syn.config1()
    os_ = oracle.OracleSpec(spec)
    data = np.load(os.path.join(HERE, "config1_data.npy"))
    q = syn.config4_draws(1)[0]
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
        assert np.array_equal(np.array(out["params"]), q)
    t0 = time.time()
    if "loglike" not in out:
        out.update(params=q.tolist(), slots=list(syn.GRAD_SLOTS), loglike=oracle.loglike(os_, q, data))
    for s in STEPS:
        key = "fd_%g" % s
        if key in out:
            continue
        g = oracle.fd_gradient(os_, q, data, syn.GRAD_SLOTS, rel_step=s)
        out[key] = g.tolist()
        print(s, g.tolist(), "%.0f s" % (time.time() - t0), flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
    for s in CHAIN_STEPS:
        key = "fdc_%g" % s
        if key in out:
            continue
        g = oracle.fd_gradient_counts(os_, q, data, syn.GRAD_SLOTS, rel_step=s)
        out[key] = g.tolist()
        print("chain", s, g.tolist(), "%.0f s" % (time.time() - t0), flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
