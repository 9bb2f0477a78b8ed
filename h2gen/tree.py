"""Cluster tree over the voxels (Sec. III.A).

The computational domain is split recursively until a cluster holds at most
`leaf_size` voxels.  The paper splits into two balanced halves; on voxel boxes
the tree here splits a box at the midpoint (first half ceil(n/2)) of every axis
whose extent is at least longest/sqrt(2).  That gives 8 children on cubes (an
octree), 4 on 2:1 slabs and 2 on rods, all balanced.

Clusters are numbered breadth first (all clusters of a level are contiguous,
and the children of one cluster are contiguous).  Each cluster owns the
contiguous range [begin, end) of tree positions; `perm[p]` is the original
(C-order) voxel index at tree position p.  Inside a leaf, voxels follow the
C order of the leaf's box.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class ClusterTree:
    shape: tuple
    leaf_size: int
    perm: np.ndarray         # (n_vox,) int64  tree position -> voxel index
    coords: np.ndarray       # (n_vox, 3) int64 integer coordinates at tree position
    level: np.ndarray        # (n_cl,) int32
    parent: np.ndarray       # (n_cl,) int32 (-1 for root)
    begin: np.ndarray        # (n_cl,) int64
    end: np.ndarray          # (n_cl,) int64
    first_child: np.ndarray  # (n_cl,) int32 (-1 for leaves)
    nchild: np.ndarray       # (n_cl,) int32
    lo: np.ndarray           # (n_cl, 3) int64 box lower corner (voxel index)
    hi: np.ndarray           # (n_cl, 3) int64 box upper corner (exclusive)

    @property
    def n_clusters(self) -> int:
        return int(self.level.shape[0])

    @property
    def n_vox(self) -> int:
        return int(self.perm.shape[0])

    @property
    def is_leaf(self) -> np.ndarray:
        return self.nchild == 0

    @property
    def depth(self) -> int:
        return int(self.level.max())

    def size(self, c) -> np.ndarray:
        return self.end[c] - self.begin[c]

    def children(self, c: int) -> range:
        f = int(self.first_child[c])
        return range(f, f + int(self.nchild[c])) if f >= 0 else range(0)

    def ancestors(self, c: int):
        out = []
        p = int(self.parent[c])
        while p >= 0:
            out.append(p)
            p = int(self.parent[p])
        return out

    def leaves(self) -> np.ndarray:
        return np.nonzero(self.nchild == 0)[0]


def _split_box(lo, hi):
    ext = hi - lo
    longest = ext.max()
    axes = [a for a in range(3) if ext[a] >= 2 and ext[a] * ext[a] * 2 >= longest * longest]
    parts = []
    for a in range(3):
        if a in axes:
            mid = lo[a] + (ext[a] + 1) // 2
            parts.append([(lo[a], mid), (mid, hi[a])])
        else:
            parts.append([(lo[a], hi[a])])
    kids = []
    for px in parts[0]:
        for py in parts[1]:
            for pz in parts[2]:
                clo = np.array([px[0], py[0], pz[0]], dtype=np.int64)
                chi = np.array([px[1], py[1], pz[1]], dtype=np.int64)
                kids.append((clo, chi))
    return kids


def build_tree(shape, leaf_size: int = 64) -> ClusterTree:
    shape = tuple(int(s) for s in shape)
    nx, ny, nz = shape
    levels, parents, lows, highs, begins, ends = [], [], [], [], [], []
    first_child, nchild = [], []
    lows.append(np.zeros(3, np.int64))
    highs.append(np.array(shape, np.int64))
    levels.append(0)
    parents.append(-1)
    begins.append(0)
    ends.append(nx * ny * nz)
    frontier = [0]
    while frontier:
        nxt = []
        for c in frontier:
            lo, hi = lows[c], highs[c]
            n = int(np.prod(hi - lo))
            if n <= leaf_size:
                first_child.append((c, -1, 0))
                continue
            kids = _split_box(lo, hi)
            start = len(levels)
            pos = begins[c]
            for clo, chi in kids:
                m = int(np.prod(chi - clo))
                levels.append(levels[c] + 1)
                parents.append(c)
                lows.append(clo)
                highs.append(chi)
                begins.append(pos)
                ends.append(pos + m)
                pos += m
                nxt.append(len(levels) - 1)
            first_child.append((c, start, len(kids)))
        frontier = nxt
    ncl = len(levels)
    fc = np.full(ncl, -1, np.int32)
    nc = np.zeros(ncl, np.int32)
    for c, f, k in first_child:
        fc[c] = f
        nc[c] = k
    lo = np.array(lows, np.int64)
    hi = np.array(highs, np.int64)
    begin = np.array(begins, np.int64)
    end = np.array(ends, np.int64)
    perm = np.empty(nx * ny * nz, np.int64)
    coords = np.empty((nx * ny * nz, 3), np.int64)
    for c in np.nonzero(nc == 0)[0]:
        bx = [np.arange(lo[c, a], hi[c, a]) for a in range(3)]
        gx, gy, gz = np.meshgrid(*bx, indexing="ij")
        cc = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
        coords[begin[c]:end[c]] = cc
        perm[begin[c]:end[c]] = (cc[:, 0] * ny + cc[:, 1]) * nz + cc[:, 2]
    return ClusterTree(shape, leaf_size, perm, coords,
                       np.array(levels, np.int32), np.array(parents, np.int32),
                       begin, end, fc, nc, lo, hi)
