"""Write the central finite differences of the FP64 oracle's FMM energy for
the differentiation workload (2^19 uniform +-1 charges, depth 6, p = 8).

Calls only the CPU oracle (oracle/); nothing here comes from the GPU library.
Output: adjoint_fd.json with
  * 64 coordinate samples (particle, axis): (E(x + h e) - E(x - h e)) / 2h at
    h = 1e-4 and at h / 2, each through oracle.fmm_probe, which evaluates that
    difference of the FMM energy as q_i (phi'(x_i + h e) - phi'(x_i - h e)) / 2h
    with the tree and expansions of the unmoved system (exact for the FMM's
    symmetric energy form; pinned against two full oracle evaluations per
    difference in tests/test_oracle_probe.py);
  * 64 charge samples: (E(q + h e_i) - E(q - h e_i)) / 2h, which for an energy
    quadratic in q with no self term equals phi_i exactly (no h dependence),
    taken as the oracle's phi_i.
Samples: seeded, among particles more than 2h from every face of their leaf
box (so x +- h stays in the leaf) and more than 20h from every other particle
(the O((h/r)^2) truncation of a central difference next to a charge at
distance r stays small).

    python tests/golden/make_adjoint_fd.py
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

H = 1e-4
SAMPLES = 64
SEED = 4004


def eligible(pos, depth, h, rng, want):
    u = pos * (1 << depth)
    fr = u - np.floor(u)
    face_ok = np.all((fr > 2 * h * (1 << depth)) & (fr < 1 - 2 * h * (1 << depth)), axis=1)
    cand = rng.permutation(np.nonzero(face_ok)[0])
    chosen = []
    for i in cand:
        d = pos - pos[i]
        r2 = np.einsum("ij,ij->i", d, d)
        r2[i] = np.inf
        if r2.min() > (20 * h) ** 2:
            chosen.append(int(i))
        if len(chosen) == want:
            break
    return np.array(chosen)


def main():
    wl = W.ADJOINT
    pos, q = wl.make()
    rng = np.random.default_rng(SEED)
    t0 = time.time()
    idx_x = eligible(pos, wl.depth, H, rng, SAMPLES)
    axis = rng.integers(0, 3, SAMPLES)
    fd = {}
    for tag, h in (("h", H), ("h_half", H / 2)):
        y = np.repeat(pos[idx_x], 2, axis=0)
        for k in range(SAMPLES):
            y[2 * k, axis[k]] += h
            y[2 * k + 1, axis[k]] -= h
        ph = oracle.fmm_probe(pos, q, wl.depth, wl.p, np.repeat(idx_x, 2), y)
        fd[tag] = (q[idx_x] * (ph[0::2] - ph[1::2]) / (2 * h)).tolist()
    idx_q = rng.choice(wl.n, SAMPLES, replace=False)
    phi_q, _, _ = oracle.fmm(pos, q, wl.depth, wl.p, targets=idx_q)
    out = {
        "workload": wl.name, "n": wl.n, "depth": wl.depth, "p": wl.p, "seed": wl.seed,
        "h": H, "x_index": idx_x.tolist(), "x_axis": axis.tolist(),
        "dE_dx_fd_h": fd["h"], "dE_dx_fd_h_half": fd["h_half"],
        "q_index": idx_q.tolist(), "dE_dq_fd": phi_q.tolist(),
        "oracle_seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, "adjoint_fd.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote adjoint_fd.json in {out['oracle_seconds']:.1f} s")


if __name__ == "__main__":
    main()
