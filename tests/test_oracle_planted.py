"""The oracle's pins catch plausible mistakes.

Each case copies fmm_oracle.c, plants one mistake by text substitution
(a dropped term, a wrong sign, a wrong index, a transposed operand), builds the
copy with gcc on the CPU and checks that the basis-free truncated-Taylor pin
rejects it.  The shipped oracle is never modified.
"""
import os
import subprocess

import numpy as np
import pytest

import kp_brute
import oracle
from oracle import build as obuild
from paper_2209_13121_amd import workloads as W

MUTATIONS = {
    # M2L sign (-1)^{k+l} replaced by (-1)^k
    "m2l_sign": ("L[hidx(k, l)] += (((k + l) & 1) ? -1.0 : 1.0) * acc;",
                 "L[hidx(k, l)] += ((k & 1) ? -1.0 : 1.0) * acc;"),
    # M2M without the complex conjugate on the shift harmonic
    "m2m_conj": ("acc += M[hidx(k, l)] * conj(harm_get(R, p, n - k, m - l));",
                 "acc += M[hidx(k, l)] * harm_get(R, p, n - k, m - l);"),
    # L2L with the shift vector reversed (transposed operand)
    "l2l_dir": ("regular_harmonics(cc[0] - c[0], cc[1] - c[1], cc[2] - c[2], p, R);",
                "regular_harmonics(c[0] - cc[0], c[1] - cc[1], c[2] - cc[2], p, R);"),
    # L2P gradient: x component with the wrong sign of the order shift
    "l2p_grad": ("gx += a * 0.5 * (rp - rm);", "gx += a * 0.5 * (rm - rp);"),
    # M2L irregular harmonic index m - l replaced by m + l
    "m2l_index": ("harm_get(Ih, 2 * p, n + k, m - l);", "harm_get(Ih, 2 * p, n + k, m + l);"),
    # regular-harmonic recurrence missing the r^2 term
    "reg_recur": ("- r2 * R[hidx(n - 2, m)]) /", ") /"),
    # interaction list that also keeps adjacent boxes (near pairs counted twice)
    "il_adjacent": ("if (iabs_(sx - ix) <= 1 && iabs_(sy - iy) <= 1 && iabs_(sz - iz) <= 1) continue;",
                    "if (sx == ix && sy == iy && sz == iz) continue;"),
    # P2P neighbour range one leaf short on the upper side
    "p2p_range": ("for (int az = cz - 1; az <= cz + 1; ++az) {", "for (int az = cz - 1; az <= cz; ++az) {"),
}


@pytest.fixture(scope="module")
def reference_case():
    pos, q = W.uniform_gauss(90, 5)
    phi_b, grad_b = kp_brute.fmm_brute(pos, q, 3, 3)
    return pos, q, phi_b, grad_b


def _build_variant(tmp_path, name, old, new):
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation {name} does not match the oracle source"
    path = os.path.join(tmp_path, f"oracle_{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmp_path, f"liboracle_{name}.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-fcx-limited-range", path, "-o", lib, "-lm"], check=True)
    return oracle.load_library(lib)


def test_unmutated_copy_passes(tmp_path, reference_case):
    pos, q, phi_b, grad_b = reference_case
    lib = _build_variant(str(tmp_path), "none", "#include <math.h>", "#include <math.h>")
    phi, f, _ = oracle.fmm(pos, q, 3, 3, lib=lib)
    assert np.linalg.norm(phi - phi_b) / np.linalg.norm(phi_b) < 1e-12


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, reference_case, name):
    pos, q, phi_b, grad_b = reference_case
    old, new = MUTATIONS[name]
    lib = _build_variant(str(tmp_path), name, old, new)
    phi, f, _ = oracle.fmm(pos, q, 3, 3, lib=lib)
    grad = -f / q[:, None]
    e_phi = np.linalg.norm(phi - phi_b) / np.linalg.norm(phi_b)
    e_grad = np.linalg.norm(grad - grad_b) / np.linalg.norm(grad_b)
    assert max(e_phi, e_grad) > 1e-6, (name, e_phi, e_grad)
