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

Two forms of the same product: ``HMatrix.matvec`` loops over the blocks;
``SparseHMatrix`` holds the same blocks as three sparse matrices, the dense
blocks D (N x N) and the stacked factors U (N x R) and V (N x R), R the sum
of the ranks, so that H = D + U V^T and y = D x + U (V^T x) (eq. (20) with
all blocks at once; row chunks may run on threads, each row's sum is taken
the same way either way).  ``HMatrix.from_arrays`` reads blocks in the
layout of the library's export (column-major dense blocks; U then V).

Pins (tests/test_oracle_hmatrix.py): the H product against the plain
product y = A x (relative error of the order of the ACA tolerance),
exactly low-rank blocks reproduced, linearity, the transpose identity
<y, H x> = <H^T y, x>, the symmetric kernel giving H^T x ~ H x; the sparse
form against the block loop (both products), threaded against unthreaded
(identical bits), and the array layout read back block for block.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.sparse as sp

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

    @classmethod
    def from_arrays(cls, n, perm, desc, off, values):
        """Blocks given as arrays: desc (nb, 6) = kind (0 dense, 1 low rank),
        r0, m, c0, n, rank; off[b] = first value of block b in values; a
        dense block is m x n column-major, a low-rank block U (m x rank)
        then V (n x rank), both column-major."""
        desc = np.asarray(desc, dtype=np.int64).reshape(-1, 6)
        values = np.asarray(values, dtype=np.float64)
        blocks = []
        for (kind, r0, m, c0, nn, r), o in zip(desc, np.asarray(off, dtype=np.int64)):
            r0, m, c0, nn, r, o = int(r0), int(m), int(c0), int(nn), int(r), int(o)
            if kind == 0:
                blocks.append(Block("dense", r0, m, c0, nn, D=values[o:o + m * nn].reshape(nn, m).T))
            else:
                U = values[o:o + m * r].reshape(r, m).T
                V = values[o + m * r:o + (m + nn) * r].reshape(r, nn).T
                blocks.append(Block("lr", r0, m, c0, nn, U=U, V=V))
        return cls(n, perm, blocks)

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


class SparseHMatrix:
    """The blocks of an HMatrix as H = D + U V^T with sparse D (N x N), U and
    V (N x R) in cluster order; products in user order like HMatrix's.
    threads > 1 splits the rows of each sparse product into chunks taken
    by a thread pool (scipy's sparse products release the interpreter
    lock); a row's sum does not depend on the split."""

    def __init__(self, H, threads=1):
        n = H.n
        self.n = n
        self.perm = np.asarray(H.perm, dtype=np.int64)
        self.threads = max(1, int(threads))
        dr, dc, dv = [], [], []
        ur, uc, uv = [], [], []
        vptr, vidx, vv = [np.zeros(1, dtype=np.int64)], [], []
        R = 0
        for b in H.blocks:
            if b.kind == "dense":
                i, j = np.meshgrid(np.arange(b.r0, b.r0 + b.m, dtype=np.int32),
                                   np.arange(b.c0, b.c0 + b.n, dtype=np.int32), indexing="ij")
                dr.append(i.ravel())
                dc.append(j.ravel())
                dv.append(np.asarray(b.D, dtype=np.float64).ravel())
            elif b.rank:
                i, k = np.meshgrid(np.arange(b.r0, b.r0 + b.m, dtype=np.int32),
                                   np.arange(R, R + b.rank, dtype=np.int32), indexing="ij")
                ur.append(i.ravel())
                uc.append(k.ravel())
                uv.append(np.asarray(b.U, dtype=np.float64).ravel())
                # row R + l of V^T is column l of V: columns c0 .. c0 + n of H
                vptr.append(np.full(b.rank, b.n, dtype=np.int64))
                vidx.append(np.tile(np.arange(b.c0, b.c0 + b.n, dtype=np.int32), b.rank))
                vv.append(np.asarray(b.V, dtype=np.float64).T.ravel())
                R += b.rank
        self.R = R

        def csr(rows, cols, vals, shape):
            if not rows:
                return sp.csr_matrix(shape)
            return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                 shape=shape).tocsr()
        self.D = csr(dr, dc, dv, (n, n))
        self.U = csr(ur, uc, uv, (n, max(R, 1)))
        if R:
            self.Vt = sp.csr_matrix((np.concatenate(vv), np.concatenate(vidx), np.cumsum(np.concatenate(vptr))),
                                    shape=(R, n))
        else:
            self.Vt = sp.csr_matrix((1, n))
        self._T = None                                      # (D^T, U^T, V), built on first use
        self._chunks = {}
        self._pool = ThreadPoolExecutor(self.threads) if self.threads > 1 else None

    @property
    def nnz(self):
        return self.D.nnz + self.U.nnz + self.Vt.nnz

    def _mv(self, M, x):
        if self._pool is None or M.shape[0] < 4 * self.threads:
            return M @ x
        key = id(M)
        if key not in self._chunks:
            edges = np.linspace(0, M.shape[0], 4 * self.threads + 1).astype(np.int64)
            self._chunks[key] = [M[a:b] for a, b in zip(edges[:-1], edges[1:]) if b > a]
        return np.concatenate(list(self._pool.map(lambda c: c @ x, self._chunks[key])))

    def matvec(self, x):
        x = np.asarray(x, dtype=np.float64)
        xc = x[self.perm]
        yc = self._mv(self.D, xc) + self._mv(self.U, self._mv(self.Vt, xc))
        y = np.empty_like(yc)
        y[self.perm] = yc
        return y

    def matvec_T(self, x):
        if self._T is None:
            self._T = (self.D.T.tocsr(), self.U.T.tocsr(), self.Vt.T.tocsr())
        Dt, Ut, V = self._T
        x = np.asarray(x, dtype=np.float64)
        xc = x[self.perm]
        yc = self._mv(Dt, xc) + self._mv(V, self._mv(Ut, xc))
        y = np.empty_like(yc)
        y[self.perm] = yc
        return y

    def close(self):
        if self._pool is not None:
            self._pool.shutdown()
            self._pool = None
