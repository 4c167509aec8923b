"""Independent enumeration of the cluster tree and the block tree (test
infrastructure): balanced bisection (or recursive 2-means) of the grid
points, admissibility of
eq. equ:adm on point bounding boxes (App. B.1), N_max = ceil(N / N_block).
Written from the definitions, sharing nothing with the library."""
import math

import numpy as np


def grid_points(dim, n, lo, hi):
    """Interior points in natural order (2D: index p*n + q, first coordinate slowest)."""
    h = (hi - lo) / (n + 1)
    x1 = lo + h * np.arange(1, n + 1)
    if dim == 1:
        return x1[:, None]
    X, Y = np.meshgrid(x1, x1, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], 1)


def two_means(coords):
    """Lloyd's iteration for two centres (Sec. 5.4, recursive K-means) on
    integer coordinates (rows of `coords`, Python ints so every comparison
    is exact).  Start: the first point of smallest and the first of largest
    coordinate along the longest side (ties: first axis).  A point joins
    the second centre only when strictly nearer; at most 64 passes, until
    no point moves; a pass that empties a side is dropped.  Returns a
    boolean array (True: second centre)."""
    pts = [(int(a), int(b)) for a, b in coords]
    ext = [max(p[a] for p in pts) - min(p[a] for p in pts) for a in (0, 1)]
    ax = 1 if ext[1] > ext[0] else 0
    vals = [p[ax] for p in pts]
    ia, ib = vals.index(min(vals)), vals.index(max(vals))
    cA, cB = [pts[ia], 1], [pts[ib], 1]      # (coordinate sums, count)

    def sq(p, c):
        (sx, sy), k = c
        return (k * p[0] - sx) ** 2 + (k * p[1] - sy) ** 2

    prev = None
    for _ in range(64):
        cur = [sq(p, cB) * cA[1] ** 2 < sq(p, cA) * cB[1] ** 2 for p in pts]
        if cur == prev:
            break
        if not any(cur) or all(cur):
            break
        prev = cur
        A = [p for p, c in zip(pts, cur) if not c]
        B = [p for p, c in zip(pts, cur) if c]
        cA = [(sum(p[0] for p in A), sum(p[1] for p in A)), len(A)]
        cB = [(sum(p[0] for p in B), sum(p[1] for p in B)), len(B)]
    return np.array(prev, dtype=bool)


def clusters(points, leaf, coords=None):
    """Levels of the balanced cluster tree: every cluster of a level is split
    until all leaves hold at most `leaf` points.  1D: index halving
    (floor(n/2) first); 2D: the longest box side at its midpoint (ties: the
    first axis), or, with `coords` (integer grid coordinates of the points),
    two_means of the cluster.  Each cluster is an array of natural indices
    (the order inside a cluster is kept)."""
    N, d = points.shape
    level = [np.arange(N)]
    tree = [level]
    while max(len(c) for c in level) > leaf:
        nxt = []
        for idx in level:
            if d == 1:
                h = len(idx) // 2
                nxt += [idx[:h], idx[h:]]
            elif coords is not None:
                m = ~two_means(coords[idx])
                nxt += [idx[m], idx[~m]]
            else:
                p = points[idx]
                lo, hi = p.min(0), p.max(0)
                ax = 1 if (hi[1] - lo[1]) > (hi[0] - lo[0]) else 0
                mid = 0.5 * (lo[ax] + hi[ax])
                m = p[:, ax] < mid
                nxt += [idx[m], idx[~m]]
        level = nxt
        tree.append(level)
    return tree


def blocks(points, tree, eta=1.0, n_block=4, min_lr=0):
    """Leaves of the block tree as (I, J, admissible) with I, J natural
    index arrays: a block is admissible when min(diam) <= eta dist of the
    two boxes, both clusters have at most N_max points and (min_lr, the
    fixed Taylor rank) at least min_lr points; inadmissible blocks are split
    down to the leaf level, where they are dense."""
    N = points.shape[0]
    nmax = math.ceil(N / n_block)
    box = lambda idx: (points[idx].min(0), points[idx].max(0))

    def diam(b):
        return float(np.linalg.norm(b[1] - b[0]))

    def dist(a, b):
        g = np.maximum(0, np.maximum(a[0] - b[1], b[0] - a[1]))
        return float(np.linalg.norm(g))

    depth = len(tree) - 1
    out = []
    stack = [(0, 0, 0)]
    while stack:
        lv, i, j = stack.pop()
        I, J = tree[lv][i], tree[lv][j]
        bi, bj = box(I), box(J)
        adm = i != j and min(diam(bi), diam(bj)) <= eta * dist(bi, bj)
        if adm and max(len(I), len(J)) <= nmax and min(len(I), len(J)) >= min_lr:
            out.append((I, J, True))
        elif lv == depth:
            out.append((I, J, False))
        else:
            for a in (2 * i, 2 * i + 1):
                for b in (2 * j, 2 * j + 1):
                    stack.append((lv + 1, a, b))
    return out
