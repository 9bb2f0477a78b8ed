"""Pins of the tree and block partition (P3), against a plain recursion of eq. (4)."""
import numpy as np
import pytest

from h2gen.partition import build_partition
from h2gen.tree import build_tree
from oracle.partition import box_diam, box_dist, partition as plain_partition

SHAPES = [(8, 8, 8), (12, 12, 12), (64, 4, 4), (32, 32, 4), (13, 13, 13), (9, 9, 9), (5, 17, 3)]


def _plain(tree, h):
    kids = {c: list(tree.children(c)) for c in range(tree.n_clusters)}
    boxes = {c: (tuple(tree.lo[c]), tuple(tree.hi[c])) for c in range(tree.n_clusters)}
    leaf = {c: bool(tree.nchild[c] == 0) for c in range(tree.n_clusters)}
    return plain_partition(kids, boxes, leaf, h)


@pytest.mark.parametrize("shape", SHAPES)
def test_partition_matches_plain_recursion(shape):
    tree = build_tree(shape, 64)
    p = build_partition(tree, 1.0)
    far, near = _plain(tree, 0.1)
    assert set(zip(p.far_t.tolist(), p.far_s.tolist())) == set(far)
    assert set(zip(p.near_t.tolist(), p.near_s.tolist())) == set(near)
    assert len(far) == p.n_far and len(near) == p.n_near


@pytest.mark.parametrize("shape", SHAPES)
def test_partition_covers_matrix_once(shape):
    tree = build_tree(shape, 64)
    p = build_partition(tree, 1.0)
    n = tree.n_vox
    cover = np.zeros((n, n), np.int32)
    for t, s in list(zip(p.far_t, p.far_s)) + list(zip(p.near_t, p.near_s)):
        cover[tree.begin[t]:tree.end[t], tree.begin[s]:tree.end[s]] += 1
    assert (cover == 1).all()


@pytest.mark.parametrize("shape", SHAPES)
def test_admissibility_and_leaf_level_near(shape):
    tree = build_tree(shape, 64)
    p = build_partition(tree, 1.0)
    h = 0.1
    for t, s in zip(p.far_t, p.far_s):
        assert max(box_diam(tree.lo[t], tree.hi[t], h), box_diam(tree.lo[s], tree.hi[s], h)) <= \
            box_dist(tree.lo[t], tree.hi[t], tree.lo[s], tree.hi[s], h) * (1 + 1e-12)
    for t, s in zip(p.near_t, p.near_s):
        assert tree.nchild[t] == 0 and tree.nchild[s] == 0       # inadmissible only at leaves
        assert max(box_diam(tree.lo[t], tree.hi[t], h), box_diam(tree.lo[s], tree.hi[s], h)) > \
            box_dist(tree.lo[t], tree.hi[t], tree.lo[s], tree.hi[s], h)
    # symmetric partition
    assert set(zip(p.far_t.tolist(), p.far_s.tolist())) == set(zip(p.far_s.tolist(), p.far_t.tolist()))


@pytest.mark.parametrize("shape", SHAPES)
def test_tree_structure(shape):
    tree = build_tree(shape, 64)
    n = tree.n_vox
    # perm is a permutation consistent with coords
    assert np.array_equal(np.sort(tree.perm), np.arange(n))
    nx, ny, nz = shape
    c = tree.coords
    assert np.array_equal(tree.perm, (c[:, 0] * ny + c[:, 1]) * nz + c[:, 2])
    for cl in range(tree.n_clusters):
        sz = tree.end[cl] - tree.begin[cl]
        assert sz == np.prod(tree.hi[cl] - tree.lo[cl])
        cc = c[tree.begin[cl]:tree.end[cl]]
        assert (cc >= tree.lo[cl]).all() and (cc < tree.hi[cl]).all()
        if tree.nchild[cl] == 0:
            assert sz <= 64
        else:
            kids = list(tree.children(cl))
            assert tree.begin[kids[0]] == tree.begin[cl] and tree.end[kids[-1]] == tree.end[cl]
            assert all(tree.parent[k] == cl and tree.level[k] == tree.level[cl] + 1 for k in kids)
            sizes = [tree.end[k] - tree.begin[k] for k in kids]
            assert max(sizes) <= 2 * min(sizes) + 16     # balanced halves


def test_octree_and_binary_split_counts():
    t = build_tree((64, 64, 64), 64)
    assert t.n_clusters == 4681 and len(t.leaves()) == 4096 and t.depth == 4
    assert set(t.nchild[t.nchild > 0].tolist()) == {8}
    t = build_tree((64, 4, 4), 64)
    assert set(t.nchild[t.nchild > 0].tolist()) == {2}
    t = build_tree((32, 32, 4), 64)
    assert set(t.nchild[t.nchild > 0].tolist()) == {4}
