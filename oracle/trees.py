"""Reference cluster tree and eta-admissible block cluster tree (oracle; test
infrastructure only).  The GPU builds the same trees and must match these
integer results bit for bit.

Cluster tree (Sec. 2.2): the index set is divided recursively into "two (equal
sized) sub-sets".  Reading adopted here (a geometric bisection into halves):

* a node is a contiguous range [lo, hi) of the permutation ``perm``
  (position -> original point index); its bounding box is the tight
  axis-parallel box of its points;
* every node of size s above the leaf level is split by an axis-parallel cut
  across the longer side of its box (x when the two extents are equal): the
  ceil(s/2) points that come first in the order (coordinate on that axis,
  original index) form the left son, the rest the right son;
* the tree is perfect: all leaves sit at depth D, the smallest D >= 0 with
  ceil(n / 2^D) <= n_min ("leaf"), so every leaf holds floor(n/2^D) or
  ceil(n/2^D) points;
* inside each leaf the points are kept in increasing original index, which
  makes ``perm`` a function of the point set alone.

Nodes are numbered per level: node i of level l covers sizes derived from n
only (left = ceil(s/2)), so ranges never depend on coordinates.

Block cluster tree (Sec. 2.2 and Appendix A, Eq. (stand_cond)): start at
(root, root) and keep the lower triangle (row cluster at or after the column
cluster).  A pair (t, s) with t != s is admissible -- a low-rank leaf -- when

    dist(B_t, B_s) > 0  and  min(diam(B_t), diam(B_s)) <= eta * dist(B_t, B_s)

evaluated in squared form, min(diam_t^2, diam_s^2) <= eta^2 * dist^2, with
diam^2 = ex^2 + ey^2 of the box extents and dist^2 = dx^2 + dy^2,
d_axis = max(0, lo_s - hi_t, lo_t - hi_s).  Otherwise the pair is a dense leaf
at depth D, else it is subdivided into its son pairs:
(t1,s1),(t1,s2),(t2,s1),(t2,s2) off the diagonal and (t1,t1),(t2,t1),(t2,t2)
on it.  Leaves are listed breadth first, sons in the order above.

All arithmetic is single IEEE-754 double operations (no fused multiply-add),
so the predicate is reproducible bit for bit.
"""
import numpy as np

LR = 1
DENSE = 0


def tree_depth(n, leaf):
    """Smallest D >= 0 with ceil(n / 2^D) <= leaf."""
    if n < 1 or leaf < 2:
        raise ValueError("need n >= 1 and leaf >= 2")
    D = 0
    while -(-n // (1 << D)) > leaf:
        D += 1
    return D


def node_ranges(n, D):
    """List over levels 0..D of int64 arrays (lo, hi) for the 2^l nodes."""
    levels = [np.array([[0, n]], dtype=np.int64)]
    for _ in range(D):
        prev = levels[-1]
        nxt = np.empty((2 * len(prev), 2), dtype=np.int64)
        for i, (lo, hi) in enumerate(prev):
            s = hi - lo
            mid = lo + (s + 1) // 2
            nxt[2 * i] = (lo, mid)
            nxt[2 * i + 1] = (mid, hi)
        levels.append(nxt)
    return levels


def _bbox(pts):
    return (float(pts[:, 0].min()), float(pts[:, 0].max()),
            float(pts[:, 1].min()), float(pts[:, 1].max()))


class ClusterTree:
    """Result of :func:`cluster_tree`.

    Attributes: ``n``, ``leaf``, ``depth``; ``perm`` (int64[n], position ->
    original index); ``ranges[l]`` (2^l x 2 int64 lo/hi); ``bbox[l]``
    (2^l x 4 float64: xmin, xmax, ymin, ymax); ``axis[l]`` (2^l int8 split
    axis of the level-l nodes, l < D).
    """


def cluster_tree(locs, leaf):
    locs = np.asarray(locs, dtype=np.float64)
    n = locs.shape[0]
    D = tree_depth(n, leaf)
    ranges = node_ranges(n, D)
    perm = np.arange(n, dtype=np.int64)
    bbox = []
    axes = []
    for l in range(D + 1):
        bb = np.empty((len(ranges[l]), 4))
        ax = np.zeros(len(ranges[l]), dtype=np.int8)
        for i, (lo, hi) in enumerate(ranges[l]):
            idx = perm[lo:hi]
            pts = locs[idx]
            bb[i] = _bbox(pts)
            if l == D:
                continue
            ex = bb[i, 1] - bb[i, 0]
            ey = bb[i, 3] - bb[i, 2]
            a = 0 if ex >= ey else 1
            ax[i] = a
            # order by (coordinate on the split axis, original index)
            order = np.lexsort((idx, pts[:, a]))
            perm[lo:hi] = idx[order]
        bbox.append(bb)
        axes.append(ax)
    for lo, hi in ranges[D]:
        perm[lo:hi] = np.sort(perm[lo:hi])
    t = ClusterTree()
    t.n, t.leaf, t.depth = n, leaf, D
    t.perm, t.ranges, t.bbox, t.axis = perm, ranges, bbox, axes[:D]
    return t


def admissible(bt, bs, eta2, rule="min"):
    """Squared-form admissibility of Appendix A: "min" the standard Adm_eta of
    Eq. (stand_cond), min(diam) <= eta dist; "max" its max(diam) form;
    "weak" Adm_W of Eq. (wead_adm), true for any two different clusters."""
    if rule == "weak":
        return True
    dx = max(max(0.0, bs[0] - bt[1]), bt[0] - bs[1])
    dy = max(max(0.0, bs[2] - bt[3]), bt[2] - bs[3])
    dist2 = dx * dx + dy * dy
    if not dist2 > 0.0:
        return False
    ext = bt[1] - bt[0]
    eyt = bt[3] - bt[2]
    dt = ext * ext + eyt * eyt
    exs = bs[1] - bs[0]
    eys = bs[3] - bs[2]
    ds = exs * exs + eys * eys
    return (max(dt, ds) if rule == "max" else min(dt, ds)) <= eta2 * dist2


def block_tree(tree, eta, rule="min"):
    """Leaves of the block cluster tree, breadth first.

    Returns an int64 array of rows (level, row_node, col_node, kind) with kind
    LR (admissible) or DENSE, node indices local to their level.
    """
    eta2 = float(eta) * float(eta)
    D = tree.depth
    frontier = [(0, 0)]
    out = []
    for l in range(D + 1):
        bb = tree.bbox[l]
        nxt = []
        for t, s in frontier:
            if t != s and admissible(bb[t], bb[s], eta2, rule):
                out.append((l, t, s, LR))
            elif l == D:
                out.append((l, t, s, DENSE))
            elif t == s:
                nxt += [(2 * t, 2 * t), (2 * t + 1, 2 * t), (2 * t + 1, 2 * t + 1)]
            else:
                nxt += [(2 * t, 2 * s), (2 * t, 2 * s + 1),
                        (2 * t + 1, 2 * s), (2 * t + 1, 2 * s + 1)]
        frontier = nxt
    return np.array(out, dtype=np.int64).reshape(-1, 4)
