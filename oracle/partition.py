"""Plain recursive block-cluster partition (test infrastructure).

Written directly from Sec. III.A: walk the row tree and column tree in
parallel from the roots; a pair is admissible when
max(diam t, diam s) <= eta * dist(t, s) (eq. (4)), with diam and dist taken
over the supports (the boxes covered by the clusters' voxels); otherwise the
children are checked, down to the leaves, where inadmissible pairs stay full.
One-at-a-time recursion in floating point; tiny inputs only.
"""

from __future__ import annotations

import math


def box_diam(lo, hi, h):
    return h * math.sqrt(sum((b - a) ** 2 for a, b in zip(lo, hi)))


def box_dist(lo1, hi1, lo2, hi2, h):
    s = 0.0
    for a in range(3):
        gap = max(0, lo2[a] - hi1[a], lo1[a] - hi2[a])
        s += gap * gap
    return h * math.sqrt(s)


def partition(tree_children, boxes, leaf, h, eta=1.0):
    """Return (far, near) as lists of (t, s).

    tree_children[c] -> list of children; boxes[c] -> (lo, hi); leaf[c] -> bool.
    """
    far, near = [], []

    def visit(t, s):
        lt, ht = boxes[t]
        ls, hs = boxes[s]
        if max(box_diam(lt, ht, h), box_diam(ls, hs, h)) <= eta * box_dist(lt, ht, ls, hs, h) + 1e-12 * h:
            far.append((t, s))
            return
        if leaf[t] and leaf[s]:
            near.append((t, s))
            return
        kids_t = [t] if leaf[t] else tree_children[t]
        kids_s = [s] if leaf[s] else tree_children[s]
        for a in kids_t:
            for b in kids_s:
                visit(a, b)

    visit(0, 0)
    return far, near
