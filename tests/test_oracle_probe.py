"""Pin of oracle.fmm_probe, the oracle's route to central differences of its
FMM energy in one coordinate (CPU only).

fmm_probe evaluates q_i (phi'(x_i + h e) - phi'(x_i - h e)) / 2h from the
unmoved tree.  Here it is compared with the literal central difference of the
oracle's energy, (E(x + h e) - E(x - h e)) / 2h, from two complete oracle FMM
runs per difference, and the charge differences with the potential.  The
stored differences of tests/golden/adjoint_fd.json are written through it.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2209_13121_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("depth,p", [(3, 4), (2, 6)])
def test_probe_equals_literal_energy_differences(depth, p):
    pos, q = W.uniform_pm1(3000, 77)
    h = 1e-4
    u = pos * (1 << depth)
    fr = u - np.floor(u)
    ok = np.nonzero(np.all((fr > 2 * h * (1 << depth)) & (fr < 1 - 2 * h * (1 << depth)), axis=1))[0]
    rng = np.random.default_rng(depth)
    for i in rng.choice(ok, 3, replace=False):
        a = int(rng.integers(0, 3))
        pp, pm = pos.copy(), pos.copy()
        pp[i, a] += h
        pm[i, a] -= h
        fd = (oracle.fmm(pp, q, depth, p)[2] - oracle.fmm(pm, q, depth, p)[2]) / (2 * h)
        y = np.array([pp[i], pm[i]])
        ph = oracle.fmm_probe(pos, q, depth, p, [i, i], y)
        fd_probe = q[i] * (ph[0] - ph[1]) / (2 * h)
        # the literal difference loses ~1e-16 |E| / h to cancellation
        assert abs(fd_probe - fd) <= 1e-9 * max(1.0, abs(fd))
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qm[i] -= h
        fdq = (oracle.fmm(pos, qp, depth, p)[2] - oracle.fmm(pos, qm, depth, p)[2]) / (2 * h)
        phi_i = oracle.fmm(pos, q, depth, p, targets=[i])[0][0]
        assert abs(fdq - phi_i) <= 1e-9 * max(1.0, abs(phi_i))


def test_probe_at_the_particle_is_its_potential():
    pos, q = W.uniform_gauss(2000, 78)
    idx = np.arange(0, 2000, 97)
    ph = oracle.fmm_probe(pos, q, 3, 5, idx, pos[idx])
    phi, _, _ = oracle.fmm(pos, q, 3, 5, targets=idx)
    assert np.allclose(ph, phi, rtol=1e-14, atol=1e-14 * np.abs(phi).max())


def test_probe_rejects_a_point_outside_the_leaf():
    pos, q = W.uniform_gauss(500, 79)
    y = pos[:1].copy()
    y[0, 0] = (np.floor(y[0, 0] * 8) + 1.5) / 8 if y[0, 0] < 0.8 else 0.01
    with pytest.raises(oracle.OracleError):
        oracle.fmm_probe(pos, q, 3, 4, [0], y)


def test_stored_adjoint_differences_are_consistent():
    # The stored h and h/2 differences agree to their O(h^2) truncation
    # (measured: at most 2.8e-3 of the RMS, the samples' neighbours being at
    # least 20 h away), and their Richardson combination is what the GPU test
    # compares against.
    g = json.load(open(os.path.join(HERE, "golden", "adjoint_fd.json")))
    a, b = np.array(g["dE_dx_fd_h"]), np.array(g["dE_dx_fd_h_half"])
    assert len(a) == len(g["x_index"]) == 64 and len(g["q_index"]) == 64
    rms = np.sqrt(np.mean(a * a))
    assert np.max(np.abs(a - b)) <= 1e-2 * rms
