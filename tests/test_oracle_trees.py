"""Pins of the reference cluster tree and block cluster tree (CPU only):
structural invariants, brute-force checks of every split, exact tiling of the
lower triangle and admissibility of every low-rank leaf on the point sets."""
import math

import numpy as np
import pytest

import workloads
from oracle import trees


@pytest.mark.parametrize("n,leaf", [(1, 32), (2, 2), (7, 2), (300, 16), (2000, 32), (1000, 64)])
def test_cluster_tree_invariants(n, leaf):
    locs, _ = workloads.uniform(n, seed=n)
    t = trees.cluster_tree(locs, leaf)
    D = t.depth
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    assert -(-n // (1 << D)) <= leaf
    if D > 0:
        assert -(-n // (1 << (D - 1))) > leaf
    for l in range(D + 1):
        r = t.ranges[l]
        sizes = r[:, 1] - r[:, 0]
        assert sizes.min() >= n // (1 << l) and sizes.max() <= -(-n // (1 << l))
        assert r[0, 0] == 0 and r[-1, 1] == n and np.all(r[1:, 0] == r[:-1, 1])
    for lo, hi in t.ranges[D]:
        assert np.all(np.diff(t.perm[lo:hi]) > 0)


def test_every_split_is_a_median_cut_across_the_longer_side():
    locs, _ = workloads.uniform(1500, seed=11)
    t = trees.cluster_tree(locs, 20)
    for l in range(t.depth):
        for i, (lo, hi) in enumerate(t.ranges[l]):
            pts = t.perm[lo:hi]
            P = locs[pts]
            bb = t.bbox[l][i]
            assert bb[0] == P[:, 0].min() and bb[1] == P[:, 0].max()
            assert bb[2] == P[:, 1].min() and bb[3] == P[:, 1].max()
            ax = 0 if (bb[1] - bb[0]) >= (bb[3] - bb[2]) else 1
            assert t.axis[l][i] == ax
            mid = t.ranges[l + 1][2 * i][1]
            left, right = t.perm[lo:mid], t.perm[mid:hi]
            assert len(left) == (hi - lo + 1) // 2
            kl = max((locs[j, ax], j) for j in left)
            kr = min((locs[j, ax], j) for j in right)
            assert kl < kr


def test_ties_break_by_original_index():
    # all points share one x: splits run along y with many equal values; among
    # equal coordinates the lower original index goes left
    ys = np.repeat(np.arange(5) * 0.1, 8)
    locs = np.stack([np.full(40, 0.5), ys], axis=1)
    t = trees.cluster_tree(locs, 4)
    lo, hi = t.ranges[0][0]
    mid = t.ranges[1][0][1]
    left, right = t.perm[lo:mid], t.perm[mid:hi]
    assert t.axis[0][0] == 1
    kl = max((locs[j, 1], j) for j in left)
    kr = min((locs[j, 1], j) for j in right)
    assert kl < kr and kl[0] == kr[0]   # the cut falls inside a tie
    t2 = trees.cluster_tree(locs, 4)
    assert np.array_equal(t.perm, t2.perm)


def _brute_block_leaves(t, eta):
    """Recursive statement of the block-tree rule, written independently."""
    out = []

    def bbox(l, i):
        lo, hi = t.ranges[l][i]
        P = t._locs[t.perm[lo:hi]]
        return P[:, 0].min(), P[:, 0].max(), P[:, 1].min(), P[:, 1].max()

    def rec(l, a, b):
        ba, bb = bbox(l, a), bbox(l, b)
        dx = max(0.0, bb[0] - ba[1], ba[0] - bb[1])
        dy = max(0.0, bb[2] - ba[3], ba[2] - bb[3])
        dist = math.hypot(dx, dy)
        diam = min(math.hypot(ba[1] - ba[0], ba[3] - ba[2]),
                   math.hypot(bb[1] - bb[0], bb[3] - bb[2]))
        if a != b and dist > 0 and diam <= eta * dist * (1 + 1e-12):
            out.append((l, a, b, trees.LR))
        elif l == t.depth:
            out.append((l, a, b, trees.DENSE))
        else:
            for c in (2 * a, 2 * a + 1):
                for d in (2 * b, 2 * b + 1):
                    if c >= d:
                        rec(l + 1, c, d)

    rec(0, 0, 0)
    return out


@pytest.mark.parametrize("n,leaf,eta", [(300, 8, 2.0), (1000, 32, 2.0), (800, 16, 1.0)])
def test_block_tree_matches_recursive_definition(n, leaf, eta):
    locs, _ = workloads.uniform(n, seed=n + 1)
    t = trees.cluster_tree(locs, leaf)
    t._locs = locs
    got = trees.block_tree(t, eta)
    ref = _brute_block_leaves(t, eta)
    assert sorted(map(tuple, got.tolist())) == sorted(ref)


@pytest.mark.parametrize("n,leaf", [(257, 8), (1200, 32)])
def test_block_leaves_tile_lower_triangle_once(n, leaf):
    locs, _ = workloads.uniform(n, seed=3)
    t = trees.cluster_tree(locs, leaf)
    leaves = trees.block_tree(t, 2.0)
    cover = np.zeros((n, n), dtype=np.int32)
    for l, a, b, kind in leaves:
        ra, rb = t.ranges[l][a], t.ranges[l][b]
        assert ra[0] >= rb[0]
        cover[ra[0]:ra[1], rb[0]:rb[1]] += 1
        if kind == trees.DENSE:
            assert l == t.depth
    low = np.tril(np.ones((n, n), dtype=bool))
    # every lower entry once; diagonal leaf blocks also hold their upper half
    assert np.all(cover[low] == 1)
    up = cover[~low]
    assert np.all((up == 0) | (up == 1))


def test_low_rank_leaves_admissible_on_point_sets():
    # bbox admissibility implies the same inequality for the point sets
    # (point diameter <= box diameter, point distance >= box distance)
    locs, _ = workloads.uniform(1500, seed=21)
    t = trees.cluster_tree(locs, 24)
    leaves = trees.block_tree(t, 2.0)
    rng = np.random.default_rng(0)
    lr = leaves[leaves[:, 3] == trees.LR]
    for l, a, b, _ in lr[rng.choice(len(lr), 60, replace=False)]:
        A = locs[t.perm[slice(*t.ranges[l][a])]]
        B = locs[t.perm[slice(*t.ranges[l][b])]]
        dA = np.sqrt(((A[:, None] - A[None]) ** 2).sum(-1)).max()
        dB = np.sqrt(((B[:, None] - B[None]) ** 2).sum(-1)).max()
        dist = np.sqrt(((A[:, None] - B[None]) ** 2).sum(-1)).min()
        assert dist > 0 and min(dA, dB) <= 2.0 * dist


def test_tree_depends_only_on_point_set():
    # relabelling the input points gives the same clusters (as point sets)
    locs, _ = workloads.uniform(700, seed=4)
    p = np.random.default_rng(1).permutation(700)
    t1 = trees.cluster_tree(locs, 16)
    t2 = trees.cluster_tree(locs[p], 16)
    for (lo, hi) in t1.ranges[t1.depth]:
        s1 = {tuple(locs[j]) for j in t1.perm[lo:hi]}
        s2 = {tuple(locs[p][j]) for j in t2.perm[lo:hi]}
        assert s1 == s2
    b1 = trees.block_tree(t1, 2.0)
    b2 = trees.block_tree(t2, 2.0)
    assert np.array_equal(b1, b2)


def test_duplicate_points_do_not_break_the_tree():
    locs = np.repeat(np.array([[0.3, 0.3], [0.7, 0.2]]), 50, axis=0)
    t = trees.cluster_tree(locs, 8)
    assert np.array_equal(np.sort(t.perm), np.arange(100))
    leaves = trees.block_tree(t, 2.0)
    assert len(leaves) > 0


# ---------------------------------------------------------------- admissibility variants
@pytest.mark.parametrize("rule", ["min", "max", "weak"])
def test_variant_block_trees_tile_lower_triangle(rule):
    n, leaf = 900, 16
    locs, _ = workloads.uniform(n, seed=5)
    t = trees.cluster_tree(locs, leaf)
    leaves = trees.block_tree(t, 2.0, rule)
    cover = np.zeros((n, n), dtype=np.int32)
    for l, a, b, kind in leaves:
        ra, rb = t.ranges[l][a], t.ranges[l][b]
        cover[ra[0]:ra[1], rb[0]:rb[1]] += 1
        if kind == trees.DENSE:
            assert l == t.depth and a == b or rule != "weak"
    low = np.tril(np.ones((n, n), dtype=bool))
    assert np.all(cover[low] == 1)


def test_weak_admissibility_is_the_sibling_pattern():
    # Eq. (wead_adm): a block of two different clusters of one level is
    # admissible, so the lower triangle splits into the off-diagonal sibling
    # blocks (2i+1, 2i) of every level and the dense diagonal leaves
    locs, _ = workloads.uniform(777, seed=6)
    t = trees.cluster_tree(locs, 16)
    D = t.depth
    want = []
    frontier = [0]
    for l in range(D + 1):
        if l == D:
            want += [(l, i, i, trees.DENSE) for i in frontier]
            break
        want += [(l + 1, 2 * i + 1, 2 * i, trees.LR) for i in frontier]
        frontier = [c for i in frontier for c in (2 * i, 2 * i + 1)]
    got = trees.block_tree(t, 2.0, "weak")
    assert sorted(map(tuple, got.tolist())) == sorted(want)


def test_max_admissibility_on_point_sets_and_refines_min():
    # the max(diam) form is the stricter condition: every low-rank leaf
    # satisfies max(diam A, diam B) <= eta dist(A, B) on its point sets, and
    # every such block is also admissible in the standard (min) sense
    locs, _ = workloads.uniform(1200, seed=22)
    t = trees.cluster_tree(locs, 24)
    mx = trees.block_tree(t, 2.0, "max")
    mn = trees.block_tree(t, 2.0, "min")
    lr = mx[mx[:, 3] == trees.LR]
    assert len(lr) > 0
    for l, a, b, _ in lr:
        A = locs[t.perm[slice(*t.ranges[l][a])]]
        B = locs[t.perm[slice(*t.ranges[l][b])]]
        dA = np.sqrt(((A[:, None] - A[None]) ** 2).sum(-1)).max()
        dB = np.sqrt(((B[:, None] - B[None]) ** 2).sum(-1)).max()
        dist = np.sqrt(((A[:, None] - B[None]) ** 2).sum(-1)).min()
        assert dist > 0 and max(dA, dB) <= 2.0 * dist
        assert trees.admissible(t.bbox[l][a], t.bbox[l][b], 4.0, "min")
    # the stricter rule never has fewer blocks
    assert len(mx) >= len(mn)
