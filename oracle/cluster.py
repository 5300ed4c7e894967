"""Cluster tree, admissibility and block partition (FP64, plain Python).

Paper: section 3.1.1 (binary cluster tree on element centres, admissibility
condition eq. 17 with eta = 2, reordering of the element indices by the
tree) and section 3.2 (lattice H-matrices: the tree is cut at depth L and
every pair of depth-L clusters, a lattice block, is partitioned on its own).

Readings of points the paper leaves open:

* Split rule: bounding box of the member centres, longest extent (ties go
  to the lowest axis, x then y then z), cut at the box midpoint; members
  with coordinate < midpoint go left, the others right, keeping their
  order.  If one side would be empty, members are stably sorted along the
  axis and the first floor(size/2) go left.
* A cluster with at most ``leaf`` members is not split (``leaf`` is the
  maximum leaf size).
* diam = Euclidean diagonal of the bounding box of the centres;
  dist = Euclidean distance between the two boxes (0 when they overlap);
  eq. 17 is applied as printed, with a strict inequality.
* Lattice: the depth-L clusters must all exist (the tree is complete to
  depth L).  A lattice block that is admissible becomes one low-rank block;
  otherwise it is refined like an ordinary H-matrix block.
* Block refinement of an inadmissible pair (tau, sigma): both leaves ->
  dense; only tau a leaf -> (tau, each child of sigma); only sigma a leaf
  -> (each child of tau, sigma); else the four child pairs, in the order
  (t1,s1), (t1,s2), (t2,s1), (t2,s2).

Parity is pinned by structural invariants only (the paper's partition
figure is not available): the permutation is a bijection, leaves respect
the size bound, boxes contain their members, blocks tile the matrix
exactly once, low-rank blocks satisfy eq. 17, dense blocks pair two leaves.
"""
from __future__ import annotations

import numpy as np


class Node:
    __slots__ = ("start", "size", "lo", "hi", "children", "depth")

    def __init__(self, start, size, lo, hi, depth):
        self.start = start
        self.size = size
        self.lo = lo
        self.hi = hi
        self.children = []
        self.depth = depth

    @property
    def is_leaf(self):
        return not self.children

    def diam(self):
        d = self.hi - self.lo
        return float(np.sqrt(np.sum(d * d)))


def dist(a: Node, b: Node) -> float:
    gap = np.maximum(0.0, np.maximum(b.lo - a.hi, a.lo - b.hi))
    return float(np.sqrt(np.sum(gap * gap)))


def admissible(a: Node, b: Node, eta: float) -> bool:
    """Eq. 17: min(diam a, diam b) < eta * dist(a, b)."""
    return min(a.diam(), b.diam()) < eta * dist(a, b)


class ClusterTree:
    def __init__(self, centres, leaf):
        centres = np.asarray(centres, dtype=np.float64)
        if leaf < 1:
            raise ValueError("leaf must be >= 1")
        self.centres = centres
        self.leaf = int(leaf)
        self.perm = np.arange(centres.shape[0], dtype=np.int64)
        self.root = self._build(0, centres.shape[0], 0)

    def _build(self, start, size, depth):
        idx = self.perm[start:start + size]
        pts = self.centres[idx]
        node = Node(start, size, pts.min(axis=0), pts.max(axis=0), depth)
        if size <= self.leaf:
            return node
        ext = node.hi - node.lo
        axis = int(np.argmax(ext))                 # first maximum: lowest axis on ties
        mid = 0.5 * (node.lo[axis] + node.hi[axis])
        below = pts[:, axis] < mid
        left = idx[below]
        right = idx[~below]
        if left.size == 0 or right.size == 0:
            order = np.argsort(pts[:, axis], kind="stable")
            half = size // 2
            left = idx[order[:half]]
            right = idx[order[half:]]
        self.perm[start:start + size] = np.concatenate([left, right])
        node.children = [self._build(start, left.size, depth + 1),
                         self._build(start + left.size, right.size, depth + 1)]
        return node

    def nodes_at_depth(self, depth):
        """Clusters at ``depth`` in left-first order; raises if the tree is
        not complete to that depth."""
        level = [self.root]
        for d in range(depth):
            nxt = []
            for nd in level:
                if nd.is_leaf:
                    raise ValueError(f"cluster tree is not complete to depth {depth} "
                                     f"(a leaf of size {nd.size} sits at depth {d})")
                nxt.extend(nd.children)
            level = nxt
        return level

    def leaves(self):
        out = []
        stack = [self.root]
        while stack:
            nd = stack.pop()
            if nd.is_leaf:
                out.append(nd)
            else:
                stack.extend(reversed(nd.children))
        return out


def partition(tree: ClusterTree, lattice: int, eta: float):
    """Block partition of the lattice H-matrix.

    Returns a list of (kind, row_node, col_node, lattice_row, lattice_col)
    with kind 'lr' (admissible) or 'dense', in lattice row-major order and,
    inside each lattice block, in depth-first refinement order.
    """
    if lattice < 1 or (lattice & (lattice - 1)) != 0:
        raise ValueError("lattice must be a power of two")
    depth = lattice.bit_length() - 1
    lat = tree.nodes_at_depth(depth)
    blocks = []

    def refine(t, s, li, lj):
        if admissible(t, s, eta):
            blocks.append(("lr", t, s, li, lj))
        elif t.is_leaf and s.is_leaf:
            blocks.append(("dense", t, s, li, lj))
        elif t.is_leaf:
            for sc in s.children:
                refine(t, sc, li, lj)
        elif s.is_leaf:
            for tc in t.children:
                refine(tc, s, li, lj)
        else:
            for tc in t.children:
                for sc in s.children:
                    refine(tc, sc, li, lj)

    for li, t in enumerate(lat):
        for lj, s in enumerate(lat):
            refine(t, s, li, lj)
    return blocks
