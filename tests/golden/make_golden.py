"""Writes stored expected values for the parity tests from the CPU oracle
only (no GPU code is imported). Usage: python tests/golden/make_golden.py medium

medium_eigs.json: the 10 lowest eigenvalues of the medium contracted matrix
(30 target orbitals, N = 10, 4 symmetries x 500 dets x 5 states, 150
continuum orbitals per irrep, 5000 L2; D = 8000), from the oracle's full
matrix and LAPACK (numpy.linalg.eigh)."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main(name):
    inst = synth.CONFIGS[name]()
    t0 = time.time()
    H = oracle.Oracle(inst).build()
    t1 = time.time()
    asym = float(np.abs(H - H.T).max())
    w = np.linalg.eigvalsh(H)
    t2 = time.time()
    out = {
        "config": name, "seed": inst.seed, "dim": int(inst.dim()),
        "lowest": [float(x) for x in w[:20]],
        "spectral_radius": float(np.abs(w).max()),
        "max_asymmetry": asym,
        "oracle_build_seconds": t1 - t0, "oracle_threads": oracle.num_threads(),
        "eigh_seconds": t2 - t1,
        "source": "tests/golden/make_golden.py (oracle/ only)",
    }
    with open(os.path.join(HERE, f"{name}_eigs.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "medium")
