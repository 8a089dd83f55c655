"""Independent count of the adaptive octree's integer statistics (CPU pin).

The adaptive tree and its four lists are rebuilt here from their definitions
(Cheng, Greengard & Rokhlin, J. Comput. Phys. 155:468 (1999), sec. 4), by
brute force over every pair of boxes, with NumPy set arithmetic and none of
the oracle's recursive descents:

  * a box holding more than leaf_max particles is divided into its 8 children
    while its level is below the depth cap; all 8 children exist;
  * two boxes touch when their closed cubes intersect;
  * U(b), b a leaf: the leaves touching b (b included);
  * V(b), b of level >= 2: the boxes of b's level whose parent touches b's
    parent and which do not touch b;
  * W(b), b a leaf: the boxes finer than b that do not touch b but whose
    parent does;
  * X(b): the leaves coarser than b that touch b's parent but not b.

Only the leaf-cell rule of the quantisation (floor of the scaled offset,
clamped) is shared with the method, written out again here.
"""
import numpy as np


def leaf_cells(pos, depth, lo, side):
    """Leaf cell per axis: floor(((x - lo) / side) 2^depth), clamped."""
    pos = np.asarray(pos, dtype=np.float64)
    if side <= 0:
        lo = pos.min(axis=0)
        side = float((pos.max(axis=0) - lo).max())
        if side == 0.0:
            side = 1.0
    lo = np.asarray(lo, dtype=np.float64)
    c = np.floor(((pos - lo) / side) * float(1 << depth)).astype(np.int64)
    return np.clip(c, 0, (1 << depth) - 1)


def build_boxes(cells, leaf_max, cap):
    """Boxes as arrays: level, coords (int64, 3), count, divided flag, parent index."""
    level, coord, count, parent = [0], [np.zeros(3, dtype=np.int64)], [len(cells)], [-1]
    divided = []
    frontier = [0]
    lvl = 0
    while frontier:
        nxt = []
        for b in frontier:
            div = count[b] > leaf_max and lvl < cap
            divided.append((b, div))
            if not div:
                continue
            sub = cells >> (cap - lvl - 1)
            for ch in range(8):
                c = 2 * coord[b] + np.array([(ch >> 2) & 1, (ch >> 1) & 1, ch & 1])
                inside = np.all(sub == c, axis=1)
                level.append(lvl + 1)
                coord.append(c)
                count.append(int(inside.sum()))
                parent.append(b)
                nxt.append(len(level) - 1)
        frontier = nxt
        lvl += 1
    div = np.zeros(len(level), dtype=bool)
    for b, d in divided:
        div[b] = d
    return (np.array(level), np.array(coord), np.array(count, dtype=np.int64), div,
            np.array(parent))


def touch_matrix(la, ca, lb, cb):
    """touch[i, j]: closed cubes of box i (levels la, coords ca) and box j intersect."""
    f = np.maximum(la[:, None], lb[None, :])
    sa, sb = f - la[:, None], f - lb[None, :]
    ok = np.ones((len(la), len(lb)), dtype=bool)
    for k in range(3):
        alo = ca[:, None, k] << sa
        ahi = (ca[:, None, k] + 1) << sa
        blo = cb[None, :, k] << sb
        bhi = (cb[None, :, k] + 1) << sb
        ok &= ~((alo > bhi) | (blo > ahi))
    return ok


def tree_stats(pos, leaf_max, cap, lo=(0.0, 0.0, 0.0), side=1.0):
    """The nine statistics the oracle and the library report, by brute force."""
    cells = leaf_cells(pos, cap, lo, side)
    level, coord, count, div, parent = build_boxes(cells, leaf_max, cap)
    nb = len(level)
    leaf = ~div
    T = touch_matrix(level, coord, level, coord)
    # U: leaves touching each leaf
    U = T & leaf[None, :] & leaf[:, None]
    u = int(U.sum())
    p2p = int((count[:, None] * count[None, :] * U).sum()) - len(cells)
    # V: same level, parents touch, boxes do not
    par = np.where(parent >= 0, parent, 0)
    Tpar = T[np.ix_(par, par)]
    same = level[:, None] == level[None, :]
    V = same & Tpar & ~T & (level[:, None] >= 2) & (parent[None, :] >= 0)
    v = int(V.sum())
    m2l = int((V & (count[:, None] > 0) & (count[None, :] > 0)).sum())
    # W: for leaf b, boxes c finer than b, not touching b, whose parent touches b
    Tbp = T[:, par] & (parent[None, :] >= 0)
    W = leaf[:, None] & (level[None, :] > level[:, None]) & ~T & Tbp
    w = int(W.sum())
    # X: for box b, leaves c coarser than b touching b's parent, not touching b
    Tpb = T[par, :] & (parent[:, None] >= 0)
    X = (level[:, None] >= 2) & leaf[None, :] & (level[None, :] < level[:, None]) & Tpb & ~T
    x = int(X.sum())
    return {"boxes": nb, "leaves": int(leaf.sum()), "deepest": int(level.max()), "u": u, "v": v,
            "w": w, "x": x, "p2p_pairs": p2p, "m2l_pairs": m2l}
