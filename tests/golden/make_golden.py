"""Write the stored oracle values the GPU tests compare against at full size.

Calls only the CPU oracle (oracle/) on the seeded workloads; nothing here
comes from the GPU library.  Output: headline_oracle.json with the FP64 FMM
energy of the 2^20-particle headline workload (uniform positions, Gaussian
charges, depth 6, p = 8), the ~1 minute an 8-core host needs for it.

    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2209_13121_amd import workloads as W  # noqa: E402


def main():
    out = {}
    for wl in (W.HEADLINE,):
        pos, q = wl.make()
        t = time.time()
        phi, force, energy = oracle.fmm(pos, q, wl.depth, wl.p)
        dt = time.time() - t
        out[wl.name] = {
            "n": wl.n, "depth": wl.depth, "p": wl.p, "seed": wl.seed, "charges": wl.charges,
            "energy": energy,
            "sum_q_phi_abs": float(np.abs(q * phi).sum()),
            "force_rms": float(np.sqrt((force**2).sum(axis=1).mean())),
            "phi_rms": float(np.sqrt((phi**2).mean())),
            "oracle_seconds": dt, "oracle_threads": os.cpu_count(),
        }
        print(wl.name, out[wl.name], flush=True)
    with open(os.path.join(HERE, "headline_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
