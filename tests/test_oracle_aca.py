"""Pins for oracle.aca (section 3.1.2, eqs. 18-19)."""
import numpy as np
import pytest

from oracle.aca import aca
from oracle.cluster import ClusterTree, partition
from oracle.greens import CoplanarRectGeometry
from synth import config_fault
from synth.faults import MU, NU


@pytest.mark.parametrize("m,n,r", [(40, 30, 1), (50, 70, 4), (64, 64, 9)])
def test_exact_low_rank_recovered(m, n, r):
    rng = np.random.default_rng(m + n + r)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    fac = aca(lambda i: A[i], lambda j: A[:, j], m, n, 1e-12)
    assert fac is not None
    U, V = fac
    assert U.shape[1] <= r + 1
    assert np.linalg.norm(A - U @ V.T) <= 1e-12 * np.linalg.norm(A)


def test_zero_block_has_rank_zero():
    A = np.zeros((20, 30))
    U, V = aca(lambda i: A[i], lambda j: A[:, j], 20, 30, 1e-6)
    assert U.shape == (20, 0) and V.shape == (30, 0)


def test_full_rank_falls_back_to_dense():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((12, 12))
    assert aca(lambda i: A[i], lambda j: A[:, j], 12, 12, 1e-10) is None
    # a max_rank below the needed rank also forces the dense fallback
    B = rng.standard_normal((40, 5)) @ rng.standard_normal((5, 40))
    assert aca(lambda i: B[i], lambda j: B[:, j], 40, 40, 1e-12, max_rank=2) is None


def test_kernel_blocks_error_and_rank():
    """On the admissible blocks of a planar fault, the Frobenius error of
    the cross approximation against the explicit block is of the order of
    the tolerance, and the rank is close to the optimal (SVD) rank."""
    f = config_fault("dip30_48x24")
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    t = ClusterTree(g.centres, 16)
    eps = 1e-6
    ratios, excess = [], []
    for kind, tau, sig, _, _ in partition(t, 4, 2.0):
        if kind != "lr":
            continue
        rows = t.perm[tau.start:tau.start + tau.size]
        cols = t.perm[sig.start:sig.start + sig.size]
        A = g.block(rows, cols)
        fac = aca(lambda i: g.entry_row(rows[i], cols), lambda j: g.entry_col(rows, cols[j]),
                  len(rows), len(cols), eps)
        if fac is None:
            continue
        U, V = fac
        err = np.linalg.norm(A - U @ V.T) / np.linalg.norm(A)
        ratios.append(err / eps)
        s = np.linalg.svd(A, compute_uv=False)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])      # tail[k] = ||A - A_k||_F
        k_opt = int(np.argmax(tail <= err * np.linalg.norm(A))) if np.any(tail <= err * np.linalg.norm(A)) else len(s)
        excess.append(U.shape[1] - k_opt)
    ratios = np.array(ratios)
    assert len(ratios) > 50
    assert np.quantile(ratios, 0.99) < 10.0
    assert ratios.max() < 100.0
    assert np.median(excess) <= 3
