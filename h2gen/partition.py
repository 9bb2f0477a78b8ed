"""Block-cluster partition under strong admissibility (Sec. III.A, eq. (4)).

Starting from (root, root), a pair (t, s) is admissible when
max(diam(t), diam(s)) <= eta * dist(t, s).  Admissible pairs become far
blocks; inadmissible pairs of two leaves become near (dense) blocks; other
inadmissible pairs are refined into their children.  When one side is a leaf
only the other side is refined.

diam and dist are taken over the support of a cluster, the closed union of
its voxel cubes, which is the box [lo*h, hi*h]: diam is the box diagonal and
dist the Euclidean distance between boxes (0 when they touch).  Both are
compared in squared integer voxel units, so the test is exact for eta = 1.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .tree import ClusterTree


@dataclass
class Partition:
    eta: float
    far_t: np.ndarray   # (n_far,) int32, sorted by (level(t), t, s)
    far_s: np.ndarray
    near_t: np.ndarray  # (n_near,) int32, sorted by (t, s)
    near_s: np.ndarray

    @property
    def n_far(self) -> int:
        return int(self.far_t.shape[0])

    @property
    def n_near(self) -> int:
        return int(self.near_t.shape[0])


def admissible(tree: ClusterTree, t: np.ndarray, s: np.ndarray, eta: float) -> np.ndarray:
    ext_t = tree.hi[t] - tree.lo[t]
    ext_s = tree.hi[s] - tree.lo[s]
    d2t = (ext_t * ext_t).sum(-1)
    d2s = (ext_s * ext_s).sum(-1)
    gap = np.maximum(0, np.maximum(tree.lo[s] - tree.hi[t], tree.lo[t] - tree.hi[s]))
    dist2 = (gap * gap).sum(-1)
    lhs = np.maximum(d2t, d2s).astype(np.float64)
    return lhs <= (eta * eta) * dist2.astype(np.float64)


def build_partition(tree: ClusterTree, eta: float = 1.0) -> Partition:
    far_t, far_s, near_t, near_s = [], [], [], []
    t = np.zeros(1, np.int64)
    s = np.zeros(1, np.int64)
    leaf = tree.nchild == 0
    while t.size:
        adm = admissible(tree, t, s, eta)
        far_t.append(t[adm])
        far_s.append(s[adm])
        t, s = t[~adm], s[~adm]
        lt, ls = leaf[t], leaf[s]
        both = lt & ls
        near_t.append(t[both])
        near_s.append(s[both])
        nt, ns = [], []
        # only the column side splits
        m = lt & ~ls
        if m.any():
            tt, ss = t[m], s[m]
            k = tree.nchild[ss]
            nt.append(np.repeat(tt, k))
            ns.append(np.concatenate([np.arange(tree.first_child[x], tree.first_child[x] + tree.nchild[x])
                                      for x in ss]))
        m = ~lt & ls
        if m.any():
            tt, ss = t[m], s[m]
            k = tree.nchild[tt]
            ns.append(np.repeat(ss, k))
            nt.append(np.concatenate([np.arange(tree.first_child[x], tree.first_child[x] + tree.nchild[x])
                                      for x in tt]))
        m = ~lt & ~ls
        if m.any():
            tt, ss = t[m], s[m]
            kt, ks = tree.nchild[tt].astype(np.int64), tree.nchild[ss].astype(np.int64)
            cnt = kt * ks
            rep_t = np.repeat(tt, cnt)
            rep_s = np.repeat(ss, cnt)
            # local index within each product block
            off = np.repeat(np.cumsum(cnt) - cnt, cnt)
            loc = np.arange(cnt.sum()) - off
            ksr = np.repeat(ks, cnt)
            nt.append(tree.first_child[rep_t] + loc // ksr)
            ns.append(tree.first_child[rep_s] + loc % ksr)
        t = np.concatenate(nt).astype(np.int64) if nt else np.zeros(0, np.int64)
        s = np.concatenate(ns).astype(np.int64) if ns else np.zeros(0, np.int64)
    ft = np.concatenate(far_t)
    fs = np.concatenate(far_s)
    o = np.lexsort((fs, ft, tree.level[ft]))
    nt_ = np.concatenate(near_t)
    ns_ = np.concatenate(near_s)
    o2 = np.lexsort((ns_, nt_))
    return Partition(eta, ft[o].astype(np.int32), fs[o].astype(np.int32),
                     nt_[o2].astype(np.int32), ns_[o2].astype(np.int32))
