#!/usr/bin/env python3
"""Write the expected values of the full-size 20-qubit workload (10 spatial
orbitals, 5 alpha + 5 beta electrons, all 875 spin-conserving UCCSD factors,
theta ~ N(0, 0.02), threshold 0) with the CPU oracle only.

    python tests/golden/make_oracle_fixtures.py

Output: tests/golden/q20_oracle.json with the FP64 energy, the full adjoint
gradient (pruning decisions frozen; exact at threshold 0), the size of the
final state and the amplitudes of 256 seeded sample determinants.  Every
number comes from oracle/ (std::map FP64 reference); the inputs come from the
seeded generator."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2301_05726_amd import synth  # noqa: E402


def main():
    wl = synth.WORKLOADS["q20"]
    p = synth.make_problem(wl, batch=1)
    nq = wl.n_qubits
    d, a, nc, du = oracle.apply_ucc(nq, [p.hf], [1.0], p.exc, p.theta[0], wl.threshold)
    E, g, _ = oracle.energy_and_grad(nq, [p.hf], [1.0], p.exc, p.theta[0], wl.threshold, p.h1, p.h2)
    rng = np.random.default_rng(4242)
    idx = np.sort(rng.choice(len(d), size=256, replace=False))
    out = {
        "what": "oracle FP64 results of the full 20-qubit workload (seeded inputs)",
        "workload": wl.name,
        "n_qubits": nq,
        "n_factors": int(p.exc.shape[0]),
        "threshold": wl.threshold,
        "energy": float(E),
        "grad": [float(x) for x in g],
        "n_det": int(len(d)),
        "det_updates": int(du),
        "sample_dets": [int(x) for x in np.asarray(d)[idx]],
        "sample_amps": [float(x) for x in np.asarray(a)[idx]],
    }
    path = os.path.join(HERE, "q20_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: E={E:.12f} N={len(d)}")


if __name__ == "__main__":
    main()
