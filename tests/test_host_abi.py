"""Host-side checks of the C ABI (no GPU needed): every symbol the header
declares is exported, the cluster/block trees match an independent
enumeration from the admissibility definition, and invalid descriptors are
rejected with HLEVY_ERR_INVALID_ARG."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hlevy.h")
LIB = os.path.join(ROOT, "paper_1812_08324_amd", "libhlevy.so")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hlevy_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def H():
    if not os.path.exists(LIB):
        pytest.skip("libhlevy.so not built")
    from paper_1812_08324_amd import hlevy
    return hlevy


def test_every_declared_symbol_is_exported(H):
    lib = ctypes.CDLL(LIB)
    names = header_functions()
    assert "hlevy_assemble" in names and "hlevy_step" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(H.EXPORTS) == set(names)
    assert H.lib.hlevy_abi_version() == 1


# ---------------------------------------------------------------------------
# independent block-tree enumeration (cluster bisection + eq. equ:adm)
# ---------------------------------------------------------------------------
def _clusters(points, leaf):
    """Balanced tree: split every cluster of a level until all leaves hold at
    most `leaf` points.  1D: index halving; 2D: longest box side at its midpoint."""
    N, d = points.shape
    level = [np.arange(N)]
    tree = [level]
    while max(len(c) for c in level) > leaf:
        nxt = []
        for idx in level:
            if d == 1:
                h = len(idx) // 2
                nxt += [idx[:h], idx[h:]]
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


def _count_blocks(points, tree, eta, nmax):
    box = lambda idx: (points[idx].min(0), points[idx].max(0))
    def diam(b):
        return float(np.linalg.norm(b[1] - b[0]))
    def dist(a, b):
        g = np.maximum(0, np.maximum(a[0] - b[1], b[0] - a[1]))
        return float(np.linalg.norm(g))
    depth = len(tree) - 1
    dense = lr = 0
    stack = [(0, 0, 0)]   # (level, i, j)
    while stack:
        lv, i, j = stack.pop()
        I, J = tree[lv][i], tree[lv][j]
        bi, bj = box(I), box(J)
        adm = i != j and min(diam(bi), diam(bj)) <= eta * dist(bi, bj)
        if adm and max(len(I), len(J)) <= nmax:
            lr += 1
        elif lv == depth:
            dense += 1
        else:
            for a in (2 * i, 2 * i + 1):
                for b in (2 * j, 2 * j + 1):
                    stack.append((lv + 1, a, b))
    return dense, lr, depth


@pytest.mark.parametrize("dim,n", [(1, 256), (1, 1000), (1, 4096), (2, 16), (2, 33), (2, 40)])
def test_block_tree_counts_match_enumeration(H, dim, n):
    lo, hi = (-1.0, 1.0) if dim == 1 else (0.0, 1.0)
    h = (hi - lo) / (n + 1)
    x1 = lo + h * np.arange(1, n + 1)
    if dim == 1:
        pts = x1[:, None]
    else:
        X, Y = np.meshgrid(x1, x1, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel()], 1)
    leaf = 64 if dim == 1 else 32
    N = pts.shape[0]
    tree = _clusters(pts, leaf)
    dense, lr, depth = _count_blocks(pts, tree, 1.0, math.ceil(N / 4))
    info = H.plan_info(H.make_problem(dim, n, lo, hi, 0.5), H.make_hparams(leaf=leaf))
    assert info["N"] == N
    assert info["depth"] == depth
    assert info["n_dense"] == dense
    assert info["n_lowrank"] == lr
    assert info["max_leaf_points"] <= leaf


def test_full_scale_counts(H):
    # 1D N = 65536, leaf 64, eta = 1, N_max = N/4: 3070 dense + 6078 low-rank leaves
    info = H.plan_info(H.make_problem(1, 65536, -1.0, 1.0, 0.75), H.make_hparams())
    assert (info["n_dense"], info["n_lowrank"], info["depth"]) == (3070, 6078, 10)


@pytest.mark.parametrize("field,value", [
    ("s", 0.0), ("s", 1.0), ("dim", 3), ("n", 1), ("a", -1.0), ("c", 0.5), ("lam", -0.1), ("r0", 0.0),
    ("lo", 2.0),
])
def test_invalid_problem_rejected(H, field, value):
    p = H.make_problem(1, 1024, -1.0, 1.0, 0.5)
    setattr(p, field, value)
    with pytest.raises(H.HlevyError) as e:
        H.plan_info(p, H.make_hparams())
    assert e.value.status == -1


@pytest.mark.parametrize("field,value", [("leaf", 8), ("leaf", 128), ("eta", 0.0), ("n_block", 0),
                                         ("aca_tol", 0.0), ("max_rank", 64)])
def test_invalid_hparams_rejected(H, field, value):
    hp = H.make_hparams()
    setattr(hp, field, value)
    with pytest.raises(H.HlevyError) as e:
        H.plan_info(H.make_problem(1, 1024, -1.0, 1.0, 0.5), hp)
    assert e.value.status == -1


def test_null_arguments_rejected(H):
    lib = H.lib
    assert lib.hlevy_plan_info(None, None, None) == -1
    assert lib.hlevy_matvec(None, None, None, None) == -1
    assert lib.hlevy_step(None, None, 1, None, None, None, None, None) == -1
    assert b"null" in lib.hlevy_last_error()
