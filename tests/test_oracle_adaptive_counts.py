"""Pin of the adaptive oracle's integer tree statistics (CPU only).

The box count, leaves, deepest level, |U|, |V|, |W|, |X| sums and the P2P and
M2L pair counts of ``oracle.fmm_adaptive`` are compared exactly with a count
made from the lists' definitions by brute force over every pair of boxes
(``tests/adaptive_count.py``, NumPy, no shared code).  The GPU tests require
the library's statistics to equal the oracle's, and the benchmark prices the
adaptive M2L from them, so these numbers need a pin of their own.
"""
import numpy as np
import pytest

import adaptive_count as AC
import oracle
from paper_2209_13121_amd import workloads as W


def clustered(n, seed, frac=0.5, width=0.04, centre=0.3):
    rng = np.random.default_rng(seed)
    m = int(n * frac)
    pos = np.concatenate([rng.random((n - m, 3)),
                          np.clip(centre + width * rng.standard_normal((m, 3)), 0.0, 1.0)])
    q = rng.standard_normal(n)
    q -= q.mean()
    return pos, q


CASES = {
    # name: (inputs, leaf_max, depth cap, cube side (0: derived))
    "blob-n400-leaf5-cap6": (lambda: clustered(400, 8), 5, 6, 1.0),
    "blob-n3000-leaf16-cap6": (lambda: clustered(3000, 21), 16, 6, 1.0),
    "blob-n5000-leaf8-cap7": (lambda: clustered(5000, 22, frac=0.7, width=0.02), 8, 7, 1.0),
    "clusters-n3000-leaf24-cap7": (lambda: W.molecular_clusters(1000, 23)[:2], 24, 7, 0.0),
    "clusters-n15000-leaf64-cap7": (lambda: W.molecular_clusters(5000, 24)[:2], 64, 7, 0.0),
    "uniform-n3000-leaf1-cap3": (lambda: W.uniform_gauss(3000, 11), 1, 3, 1.0),
    "root-leaf-n150": (lambda: clustered(150, 12), 200, 6, 1.0),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_tree_stats_match_brute_force_count(name):
    make, leaf_max, cap, side = CASES[name]
    pos, q = make()
    _, _, _, st = oracle.fmm_adaptive(pos, q, leaf_max, cap, 1, side=side)
    assert st == AC.tree_stats(pos, leaf_max, cap, side=side)


def test_count_sees_a_changed_definition():
    # The brute-force count is not blind to the lists: counting V without the
    # "parents touch" condition, or U without "touch", changes the numbers.
    pos, q = clustered(3000, 21)
    cells = AC.leaf_cells(pos, 6, (0, 0, 0), 1.0)
    level, coord, count, div, parent = AC.build_boxes(cells, 16, 6)
    T = AC.touch_matrix(level, coord, level, coord)
    same = level[:, None] == level[None, :]
    v_loose = int((same & ~T & (level[:, None] >= 2)).sum())
    st = AC.tree_stats(pos, 16, 6)
    assert v_loose > st["v"]
    leaf = ~div
    assert int((leaf[:, None] & leaf[None, :]).sum()) > st["u"]
