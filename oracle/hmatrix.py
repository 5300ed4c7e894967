"""Lattice H-matrix build and H-matrix-vector product (FP64).

Paper: section 3.1 (construction: cluster tree, partition by eq. 17, ACA
of admissible blocks by eqs. 18-19, dense storage of the rest), section
3.2 (lattice structure) and section 3.1.3, eq. (20): the product is taken
block by block, y_L += A_LM x_M for dense blocks and
y_L += g^T (h x_M) for low-rank blocks, and the full result is the sum of
all block contributions.

Indices: blocks refer to rows/columns in cluster order (positions in the
tree permutation ``perm``); user-order vectors are gathered with ``perm``
before the product and scattered back after it.

Pins (tests/test_oracle_hmatrix.py): the H product against the plain
product y = A x (relative error of the order of the ACA tolerance),
exactly low-rank blocks reproduced, linearity, the transpose identity
<y, H x> = <H^T y, x>, the symmetric kernel giving H^T x ~ H x.
"""
from __future__ import annotations

import numpy as np

from .aca import aca
from .cluster import ClusterTree, partition


class Block:
    __slots__ = ("kind", "r0", "m", "c0", "n", "D", "U", "V", "lat")

    def __init__(self, kind, r0, m, c0, n, D=None, U=None, V=None, lat=(0, 0)):
        self.kind = kind
        self.r0, self.m, self.c0, self.n = r0, m, c0, n
        self.D, self.U, self.V = D, U, V
        self.lat = lat

    @property
    def rank(self):
        return 0 if self.U is None else self.U.shape[1]

    def entries(self):
        return self.m * self.n if self.kind == "dense" else self.rank * (self.m + self.n)


class HMatrix:
    """Blocks (in cluster order) plus the permutation."""

    def __init__(self, n, perm, blocks):
        self.n = int(n)
        self.perm = np.asarray(perm, dtype=np.int64)
        self.blocks = list(blocks)

    # -- construction ------------------------------------------------------
    @classmethod
    def build(cls, geom, leaf, eta, aca_eps, lattice=1, max_rank=0, lattice_rows=None):
        """geom provides .centres, .block(rows, cols), .entry_row(i, cols),
        .entry_col(rows, j) in user order.  ``lattice_rows``: build only the
        blocks of these lattice block-rows (a sample; other rows of the
        product stay zero)."""
        tree = ClusterTree(geom.centres, leaf)
        perm = tree.perm
        blocks = []
        for kind, t, s, li, lj in partition(tree, lattice, eta):
            if lattice_rows is not None and li not in lattice_rows:
                continue
            rows = perm[t.start:t.start + t.size]
            cols = perm[s.start:s.start + s.size]
            if kind == "lr":
                fac = aca(lambda i: geom.entry_row(rows[i], cols),
                          lambda j: geom.entry_col(rows, cols[j]),
                          t.size, s.size, aca_eps, max_rank)
                if fac is not None:
                    blocks.append(Block("lr", t.start, t.size, s.start, s.size,
                                        U=fac[0], V=fac[1], lat=(li, lj)))
                    continue
            blocks.append(Block("dense", t.start, t.size, s.start, s.size,
                                D=geom.block(rows, cols), lat=(li, lj)))
        h = cls(geom.centres.shape[0], perm, blocks)
        h.tree = tree
        h.lattice = lattice
        return h

    def lattice_row_ranges(self, rows):
        """[start, end) of the given lattice block-rows in cluster order."""
        lat = self.tree.nodes_at_depth(self.lattice.bit_length() - 1)
        return [(lat[i].start, lat[i].start + lat[i].size) for i in rows]

    # -- products (eq. 20) -------------------------------------------------
    def matvec(self, x):
        """y = H x for user-order x of shape (N,) or (N, k)."""
        x = np.asarray(x, dtype=np.float64)
        xc = x[self.perm]
        yc = np.zeros_like(xc)
        for b in self.blocks:
            xs = xc[b.c0:b.c0 + b.n]
            if b.kind == "dense":
                yc[b.r0:b.r0 + b.m] += b.D @ xs
            elif b.rank:
                yc[b.r0:b.r0 + b.m] += b.U @ (b.V.T @ xs)
        y = np.empty_like(yc)
        y[self.perm] = yc
        return y

    def matvec_T(self, x):
        """y = H^T x (user order)."""
        x = np.asarray(x, dtype=np.float64)
        xc = x[self.perm]
        yc = np.zeros_like(xc)
        for b in self.blocks:
            xs = xc[b.r0:b.r0 + b.m]
            if b.kind == "dense":
                yc[b.c0:b.c0 + b.n] += b.D.T @ xs
            elif b.rank:
                yc[b.c0:b.c0 + b.n] += b.V @ (b.U.T @ xs)
        y = np.empty_like(yc)
        y[self.perm] = yc
        return y

    def to_dense(self):
        """Explicit N x N matrix represented by the blocks (small N only)."""
        A = np.zeros((self.n, self.n))
        for b in self.blocks:
            if b.kind == "dense":
                blk = b.D
            else:
                blk = b.U @ b.V.T
            A[b.r0:b.r0 + b.m, b.c0:b.c0 + b.n] = blk
        P = np.empty_like(A)
        P[np.ix_(self.perm, self.perm)] = A
        return P

    # -- statistics --------------------------------------------------------
    def stats(self):
        nd = sum(1 for b in self.blocks if b.kind == "dense")
        nl = len(self.blocks) - nd
        dense_e = sum(b.m * b.n for b in self.blocks if b.kind == "dense")
        lr_e = sum(b.rank * (b.m + b.n) for b in self.blocks if b.kind == "lr")
        ranks = [b.rank for b in self.blocks if b.kind == "lr"]
        return dict(n=self.n, n_dense=nd, n_lr=nl, dense_entries=dense_e,
                    lr_entries=lr_e, entries=dense_e + lr_e,
                    max_rank=max(ranks) if ranks else 0,
                    compression=(dense_e + lr_e) / float(self.n) ** 2)
