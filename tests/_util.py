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


def _oracle_rows_worker(args):
    """Blocks of the given lattice block-rows of a planar workload, built
    by the oracle (runs in a spawned process)."""
    name, rows = args
    sys.path.insert(0, ROOT)
    from threadpoolctl import threadpool_limits

    from oracle.greens import CoplanarRectGeometry
    from oracle.hmatrix import HMatrix
    from synth import WORKLOADS, config_fault
    from synth.faults import MU, NU
    w = WORKLOADS[name]
    f = config_fault(name)
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    with threadpool_limits(limits=1):
        H = HMatrix.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"], lattice_rows=set(rows))
    return H.perm, H.blocks


def oracle_build_parallel(name, workers=None):
    """The oracle's H-matrix of a planar workload, its lattice block-rows
    built by the oracle's own construction in separate processes (spawned:
    no GPU state is inherited) and joined; identical to a serial build (each
    block depends only on its own rows and columns, and they are put back
    in the serial order)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    from oracle.hmatrix import HMatrix
    from synth import WORKLOADS
    lat = WORKLOADS[name]["lattice"]
    workers = workers or min(16, len(os.sched_getaffinity(0)), lat)
    chunks = [tuple(range(i, lat, workers)) for i in range(workers)]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_oracle_rows_worker, [(name, c) for c in chunks]))
    perm = parts[0][0]
    assert all(np.array_equal(p, perm) for p, _ in parts)
    # a lattice pair's blocks all come from one worker, in partition order
    blocks = sorted((b for _, bl in parts for b in bl), key=lambda b: b.lat)
    return HMatrix(len(perm), perm, blocks)


def _triangle_columns(args):
    """The oracle's A and B columns of a triangle mesh (spawned process)."""
    verts, slip, cols = args
    sys.path.insert(0, ROOT)
    from oracle.triangles import TriangleGeometry
    from synth.faults import MU, NU
    return TriangleGeometry(verts, slip, MU, NU).blocks(np.arange(verts.shape[0]), cols)


def oracle_triangle_matrices(verts, slip_dir, workers=16):
    """The oracle's dense A and B of a triangle mesh (its cubature of every
    entry), the sources split over spawned processes."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(workers, len(os.sched_getaffinity(0))))
    chunks = np.array_split(np.arange(verts.shape[0]), 4 * workers)
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_triangle_columns, [(verts, slip_dir, c) for c in chunks]))
    return np.concatenate([a for a, _ in parts], axis=1), np.concatenate([b for _, b in parts], axis=1)


def _triangle_rows(args):
    verts, slip, rows, cols = args
    sys.path.insert(0, ROOT)
    from oracle.triangles import TriangleGeometry
    from synth.faults import MU, NU
    return TriangleGeometry(verts, slip, MU, NU).blocks(rows, cols)


def oracle_triangle_rows(verts, slip_dir, rows, workers=16):
    """Rows of the oracle's A and B of a triangle mesh (its cubature), the
    sources split over spawned processes."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(workers, len(os.sched_getaffinity(0))))
    rows = np.asarray(rows)
    chunks = np.array_split(np.arange(verts.shape[0]), 4 * workers)
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_triangle_rows, [(verts, slip_dir, rows, c) for c in chunks]))
    return np.concatenate([a for a, _ in parts], axis=1), np.concatenate([b for _, b in parts], axis=1)
