"""Pins for oracle.cluster (section 3.1.1, eq. 17; section 3.2 lattice).

The paper prints no partition, so these are the structural invariants any
correct cluster tree and block partition must satisfy.
"""
import numpy as np
import pytest

from oracle.cluster import ClusterTree, admissible, dist, partition
from oracle.greens import CoplanarRectGeometry
from synth import config_fault, planar_rect_fault
from synth.faults import MU, NU


def _centres(f):
    return CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU).centres


CASES = [("planar64x32", 32, 1), ("dip30_48x24", 16, 4), ("strike_37x23", 20, 2)]


@pytest.mark.parametrize("name,leaf,lattice", CASES)
def test_tree_invariants(name, leaf, lattice):
    f = config_fault(name)
    c = _centres(f)
    t = ClusterTree(c, leaf)
    assert np.array_equal(np.sort(t.perm), np.arange(f.n))
    stack = [t.root]
    total_leaf = 0
    while stack:
        nd = stack.pop()
        pts = c[t.perm[nd.start:nd.start + nd.size]]
        assert np.all(pts >= nd.lo) and np.all(pts <= nd.hi)
        if nd.is_leaf:
            assert 1 <= nd.size <= leaf
            total_leaf += nd.size
        else:
            a, b = nd.children
            assert a.start == nd.start and b.start == a.start + a.size
            assert a.size + b.size == nd.size and a.size > 0 and b.size > 0
            stack.extend(nd.children)
    assert total_leaf == f.n


@pytest.mark.parametrize("name,leaf,lattice", CASES)
def test_partition_tiles_matrix_once(name, leaf, lattice):
    f = config_fault(name)
    t = ClusterTree(_centres(f), leaf)
    blocks = partition(t, lattice, 2.0)
    cover = np.zeros((f.n, f.n), dtype=np.int32)
    for kind, tau, sig, li, lj in blocks:
        cover[tau.start:tau.start + tau.size, sig.start:sig.start + sig.size] += 1
        if kind == "lr":
            assert admissible(tau, sig, 2.0)
            assert min(tau.diam(), sig.diam()) < 2.0 * dist(tau, sig)
        else:
            assert tau.is_leaf and sig.is_leaf
            assert not admissible(tau, sig, 2.0)
    assert np.all(cover == 1)
    # lattice: every block lies inside one lattice block
    lat = t.nodes_at_depth(lattice.bit_length() - 1)
    assert len(lat) == lattice
    for kind, tau, sig, li, lj in blocks:
        L, S = lat[li], lat[lj]
        assert L.start <= tau.start and tau.start + tau.size <= L.start + L.size
        assert S.start <= sig.start and sig.start + sig.size <= S.start + S.size


def test_midpoint_split_and_ties():
    # 1D points along y: the longest box side is y, split at the midpoint
    c = np.zeros((6, 3))
    c[:, 1] = [0.0, 5.0, 1.0, 4.0, 2.0, 3.0]
    t = ClusterTree(c, 3)
    left, right = t.root.children
    assert list(t.perm[:3]) == [0, 2, 4] and list(t.perm[3:]) == [1, 3, 5]
    # identical points: median fallback puts floor(n/2) on the left
    t2 = ClusterTree(np.ones((5, 3)), 2)
    assert [ch.size for ch in t2.root.children] == [2, 3]
    # equal extents: the lowest axis (x) is cut first
    sq = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], dtype=float)
    t3 = ClusterTree(sq, 2)
    assert sorted(t3.perm[:2]) == [0, 2]


def test_admissibility_is_strict():
    c = np.array([[0.0, 0, 0], [1.0, 0, 0], [3.0, 0, 0], [4.0, 0, 0]])
    t = ClusterTree(c, 2)
    a, b = t.root.children
    # diam = 1, dist = 2: 1 < 2 * 2 admissible; with eta = 0.5: 1 < 1 is false
    assert admissible(a, b, 2.0)
    assert not admissible(a, b, 0.5)


def test_incomplete_lattice_rejected():
    f = planar_rect_fault(4, 4, 100.0, 90.0, "strike")
    t = ClusterTree(_centres(f), 8)
    with pytest.raises(ValueError):
        partition(t, 4, 2.0)
