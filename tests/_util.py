"""Shared helpers of the test-suite (test infrastructure only)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def oracle_blocks(H):
    """Oracle H-matrix -> arrays in the hmat_host_blocks layout."""
    desc, off, vals = [], [], []
    at = 0
    for b in H.blocks:
        if b.kind == "dense":
            v = b.D.T.reshape(-1)                    # column-major m x n
            desc.append([0, b.r0, b.m, b.c0, b.n, 0])
        else:
            v = np.concatenate([b.U.T.reshape(-1), b.V.T.reshape(-1)])
            desc.append([1, b.r0, b.m, b.c0, b.n, b.rank])
        off.append(at)
        vals.append(v)
        at += v.size
    return dict(n=H.n, perm=H.perm.astype(np.int32), desc=np.array(desc, dtype=np.int64),
                off=np.array(off, dtype=np.int64), values=np.concatenate(vals))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
