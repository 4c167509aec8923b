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
    assert H.lib.hlevy_abi_version() == 6


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
                                         ("aca_tol", 0.0), ("max_rank", 64), ("gather_waves", 2),
                                         ("gather_waves", 16), ("rank_bucket", 12), ("rank_bucket", 64),
                                         ("strict_rank_cap", 2)])
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


# ---------------------------------------------------------------------------
# host-side contract of the calls added with the refinement checks
# ---------------------------------------------------------------------------
def test_lowrank_block_row_limit(H):
    """Admissible blocks are limited to 16384 rows (the ACA kernel's pivot-row
    bitmap): N = 2^17 with N_max = N/4 is rejected by every entry point that
    builds the trees, and accepted once n_block keeps blocks within the limit."""
    p = H.make_problem(1, 1 << 17, -1.0, 1.0, 0.5)
    with pytest.raises(H.HlevyError) as e:
        H.plan_info(p, H.make_hparams())
    assert e.value.status == -1 and "16384" in str(e.value)
    with pytest.raises(H.HlevyError):
        H.footprint(p, H.make_hparams())
    info = H.plan_info(p, H.make_hparams(n_block=8))
    assert info["N"] == 1 << 17


def test_window_radius_must_fit_the_domain(H):
    p = H.make_problem(1, 1024, -1.0, 1.0, 0.5, r0=2.5)
    with pytest.raises(H.HlevyError) as e:
        H.plan_info(p, H.make_hparams())
    assert e.value.status == -1 and "r0" in str(e.value)


def test_server_submit_validates_like_assembly(H):
    """Submission runs the structure validation before touching the device:
    an over-limit problem is rejected at submit, not later in a poll."""
    lib = H.lib
    cfg = H.ServerConfig(0, H.PREC_MIXED, 1e-6, 1, 10, 16, 0.0)
    srv = ctypes.c_void_p()
    assert lib.hlevy_server_create(ctypes.byref(cfg), None, ctypes.byref(srv)) == 0
    try:
        rid = ctypes.c_int64()
        fake = ctypes.c_void_p(256)   # never dereferenced: validation fails first
        from workloads import lshape_mask
        for prob, hp in [(H.make_problem(1, 1 << 17, -1.0, 1.0, 0.5), H.make_hparams()),
                         (H.make_problem(1, 1024, -1.0, 1.0, 0.5, r0=3.0), H.make_hparams()),
                         (H.make_problem(2, 40, -1.0, 1.0, 0.5, mask=lshape_mask(40)), H.make_hparams())]:
            st = lib.hlevy_server_submit(srv, ctypes.byref(prob), ctypes.byref(hp), 1e-3, 10, fake, fake,
                                         ctypes.byref(rid))
            assert st == -1
        stats = H.ServerStats()
        assert lib.hlevy_server_stats_get(srv, ctypes.byref(stats)) == 0
        assert stats.submitted == 0 and stats.failed == 0 and stats.max_rel_residual == -1.0
        n = ctypes.c_int32(5)
        ids = (ctypes.c_int64 * 4)()
        assert lib.hlevy_server_take_failed(srv, ids, 4, ctypes.byref(n)) == 0 and n.value == 0
    finally:
        lib.hlevy_server_destroy(srv)


def test_server_config_rejects_nonfinite_tol(H):
    cfg = H.ServerConfig(0, H.PREC_MIXED, 1e-6, 1, 10, 16, float("nan"))
    srv = ctypes.c_void_p()
    assert H.lib.hlevy_server_create(ctypes.byref(cfg), None, ctypes.byref(srv)) == -1


def _lr_blocks(pts, tree, eta, nmax):
    """(rows, cols) of every admissible leaf of the block tree (equ:adm on
    bounding boxes, size at most nmax)."""
    out = []

    def box(idx):
        p = pts[idx]
        return p.min(0), p.max(0)

    def rec(lv, a, b):
        ia, ib = tree[lv][a], tree[lv][b]
        (la, ha), (lb, hb) = box(ia), box(ib)
        diam = min(np.linalg.norm(ha - la), np.linalg.norm(hb - lb))
        gap = np.maximum(0.0, np.maximum(la - hb, lb - ha))
        dist = np.linalg.norm(gap)
        if a != b and diam <= eta * dist and max(len(ia), len(ib)) <= nmax:
            out.append((len(ia), len(ib)))
        elif lv + 1 < len(tree):
            for i in (2 * a, 2 * a + 1):
                for j in (2 * b, 2 * b + 1):
                    rec(lv + 1, i, j)

    rec(0, 0, 0)
    return out


@pytest.mark.parametrize("dim,n,kcap", [(1, 4096, 16), (2, 48, 32)])
def test_footprint_bounds_the_stored_factors(H, dim, n, kcap):
    """hlevy_footprint covers at least the three H-matrices a factor keeps
    (G, L^{-1}, U^{-1}), each with every admissible block at its rank
    capacity, and the mixed path's FP32 copies of the inverse factors; and
    it stays within a few percent of those bytes (the rest is plans and
    vectors).  The block list comes from the independent enumeration."""
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
    lr = _lr_blocks(pts, tree, 1.0, math.ceil(N / 4))
    hp = H.make_hparams(leaf=leaf, max_rank=kcap, aca_tol=1e-8)
    prob = H.make_problem(dim, n, lo, hi, 0.5)
    info = H.plan_info(prob, hp)
    assert len(lr) == info["n_lowrank"]
    lr_entries = sum((m + k) * min(kcap, m, k) for m, k in lr)
    # G holds every block; L^{-1} and U^{-1} the lower / upper halves and both the diagonal
    diag = N * leaf   # dense diagonal leaves: at most one leaf x leaf block per leaf cluster
    g_bytes = 8 * (info["dense_entries"] + lr_entries)
    inv_bytes = 8 * (info["dense_entries"] + lr_entries + diag)
    f64 = H.footprint(prob, hp, H.PREC_FP64)
    mixed = H.footprint(prob, hp, H.PREC_MIXED)
    assert f64 >= g_bytes + 8 * (info["dense_entries"] + lr_entries)
    assert f64 <= 1.25 * (g_bytes + inv_bytes) + 64 * N
    # FP32 copies of both inverse factors on the mixed path
    assert mixed - f64 >= 4 * (info["dense_entries"] + lr_entries)


def test_autotune_cache_hit_needs_no_device(H, tmp_path):
    """A tuning cache entry for the problem's key (dimension, N rounded to a
    power of two, precision, batched) is returned as stored, without device
    work; other keys, other precisions and the single path miss it."""
    path = tmp_path / "tune.json"
    path.write_text('{"version": 1, "entries": {"d1_n13_p1_batched": {"leaf": 32, "gather_waves": 4, '
                    '"rank_bucket": 16, "seconds": 0.0125, "default_seconds": 0.015}}}\n')
    prob = H.make_problem(1, 9000, -1.0, 1.0, 0.4, lam=0.5, a=0.01, b=(0.3, 0.0))
    hp = H.make_hparams(aca_tol=1e-10, max_rank=16)
    tuned, res = H.autotune(prob, hp, 1e-3, H.PREC_MIXED, 1e-6, 100, batch=8, cache=str(path), stream=0)
    assert res["from_cache"] and (res["leaf"], res["gather_waves"], res["rank_bucket"]) == (32, 4, 16)
    assert res["seconds"] == 0.0125 and res["default_seconds"] == 0.015
    assert (tuned.leaf, tuned.gather_waves, tuned.rank_bucket) == (32, 4, 16)
    assert tuned.max_rank == 16 and tuned.aca_tol == 1e-10
    with pytest.raises(H.HlevyError) as e:      # invalid arguments are rejected before the cache
        H.autotune(prob, hp, -1.0, H.PREC_MIXED, 1e-6, 100, batch=8, cache=str(path), stream=0)
    assert e.value.status == -1


def test_gaussian_validation(H):
    """Gaussian kernel needs eps2 > 0 and the Taylor construction; taylor_rank
    needs the Gaussian kernel and at most max_rank."""
    ok = H.make_hparams(taylor_rank=10)
    with pytest.raises(H.HlevyError, match="eps2"):
        H.plan_info(H.make_problem(1, 256, -1.0, 1.0, 0.5, kernel=H.KERNEL_GAUSSIAN, eps2=0.0), ok)
    with pytest.raises(H.HlevyError, match="taylor_rank"):
        H.plan_info(H.make_problem(1, 256, -1.0, 1.0, 0.5), ok)
    with pytest.raises(H.HlevyError, match="taylor_rank"):
        H.plan_info(H.make_problem(1, 256, -1.0, 1.0, 0.5, kernel=H.KERNEL_GAUSSIAN, eps2=5.0),
                    H.make_hparams(taylor_rank=20, max_rank=16))
    with pytest.raises(H.HlevyError, match="taylor_rank > 0"):
        H.plan_info(H.make_problem(2, 40, -1.0, 1.0, 0.5, kernel=H.KERNEL_GAUSSIAN, eps2=5.0),
                    H.make_hparams(taylor_rank=0))


def test_asymmetric_kernel_validation(H):
    """The asymmetric tempered kernel (1D, and 2D tilted along the first
    axis) needs lambda_neg >= 0."""
    hp = H.make_hparams()
    H.plan_info(H.make_problem(1, 256, -1.0, 1.0, 0.5, lam=0.5, lam_neg=3.0), hp)
    assert H.plan_info(H.make_problem(2, 40, 0.0, 1.0, 0.5, lam=0.5, lam_neg=3.0), hp)["N"] == 1600
    with pytest.raises(H.HlevyError, match="lambda_neg"):
        H.plan_info(H.make_problem(1, 256, -1.0, 1.0, 0.5, lam=0.5, lam_neg=-1.0), hp)


# ---------------------------------------------------------------------------
# masked domains, 2-means clustering, variable jump index (Sec. 5.4)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,leaf,kmeans", [(16, 16, True), (30, 32, True), (40, 32, True), (40, 32, False),
                                           (60, 64, True)])
def test_lshape_tree_matches_enumeration(H, n, leaf, kmeans):
    """The L-shaped domain's cluster and block trees (recursive 2-means on
    the integer grid coordinates, or bisection) equal the independent
    enumeration of tests/blocktree.py: depth, dense and low-rank leaves."""
    from blocktree import blocks, clusters
    from workloads import lshape_mask, variable_order_lshape
    w = variable_order_lshape(n)
    g = np.flatnonzero(lshape_mask(n).reshape(-1))
    coords = np.stack([g // n, g % n], 1) if kmeans else None
    tree = clusters(w["x"], leaf, coords)
    bl = blocks(w["x"], tree)
    prob = H.make_problem(2, n, -1.0, 1.0, 0.5, mask=w["mask"], s_field=w["s"])
    info = H.plan_info(prob, H.make_hparams(leaf=leaf, cluster=H.CLUSTER_KMEANS if kmeans else H.CLUSTER_BISECT))
    assert info["N"] == w["N"] == 3 * n * n // 4
    assert info["depth"] == len(tree) - 1
    assert info["n_dense"] == sum(1 for *_, a in bl if not a)
    assert info["n_lowrank"] == sum(1 for *_, a in bl if a)
    assert info["max_leaf_points"] == max(len(c) for c in tree[-1])
    assert info["min_leaf_points"] == min(len(c) for c in tree[-1])


def test_two_means_is_a_lloyd_fixed_point():
    """Each split of the test enumeration's 2-means leaves every point with
    the nearer of the two centres (ties with the first) and both sides
    non-empty, and the first split of the L-shape separates its two arms."""
    from blocktree import two_means
    from workloads import lshape_mask
    n = 30
    g = np.flatnonzero(lshape_mask(n).reshape(-1))
    coords = np.stack([g // n, g % n], 1)
    side = two_means(coords)
    assert side.any() and not side.all()
    ca, cb = coords[~side].mean(0), coords[side].mean(0)
    da = ((coords - ca) ** 2).sum(1)
    db = ((coords - cb) ** 2).sum(1)
    assert np.all(side == (db < da))


def test_variable_order_validation(H):
    """The variable-order kernel needs one index in (0, 1) per unknown; a
    mask needs 2D; KMEANS is 2D; the server takes no mask."""
    from workloads import lshape_mask
    hp = H.make_hparams()
    mask = lshape_mask(40)
    ok = H.make_problem(2, 40, -1.0, 1.0, 0.5, mask=mask, s_field=np.full(1200, 0.5))
    assert H.plan_info(ok, hp)["N"] == 1200
    bad = H.make_problem(2, 40, -1.0, 1.0, 0.5, mask=mask, s_field=np.r_[np.full(1199, 0.5), 1.0])
    with pytest.raises(H.HlevyError, match=r"s_field\[1199\]"):
        H.plan_info(bad, hp)
    p = H.make_problem(2, 40, -1.0, 1.0, 0.5)
    p.kernel = H.KERNEL_VARIABLE_ORDER
    with pytest.raises(H.HlevyError, match="needs s_field"):
        H.plan_info(p, hp)
    with pytest.raises(H.HlevyError, match="variable-order kernel only"):
        q = H.make_problem(1, 256, -1.0, 1.0, 0.5, s_field=np.full(256, 0.5))
        q.kernel = H.KERNEL_TEMPERED
        H.plan_info(q, hp)
    with pytest.raises(H.HlevyError, match="mask needs dim 2"):
        H.plan_info(H.make_problem(1, 4, -1.0, 1.0, 0.5, mask=np.ones((4, 4))), hp)
    with pytest.raises(H.HlevyError, match="2D only"):
        H.plan_info(H.make_problem(1, 256, -1.0, 1.0, 0.5), H.make_hparams(cluster=H.CLUSTER_KMEANS))
    with pytest.raises(H.HlevyError, match="cluster must be"):
        H.plan_info(H.make_problem(1, 256, -1.0, 1.0, 0.5), H.make_hparams(cluster=2))
    few = np.zeros((40, 40), dtype=bool)
    few[0, :10] = True
    with pytest.raises(H.HlevyError, match="twice the leaf"):
        H.plan_info(H.make_problem(2, 40, -1.0, 1.0, 0.5, mask=few), hp)
